// Direct pencil-pass kernels: storage f16, transform sign -1.
#define WSFFT_IO IoF16
#define WSFFT_SIGN (-1)
#define WSFFT_FIND find_pass_f16_neg
#include "pass_inst.inc"
