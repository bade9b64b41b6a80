// Direct pencil-pass kernels: storage bf16, transform sign -1.
#define WSFFT_IO IoBF16
#define WSFFT_SIGN (-1)
#define WSFFT_FIND find_pass_bf16_neg
#include "pass_inst.inc"
