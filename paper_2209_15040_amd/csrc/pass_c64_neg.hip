// Direct pencil-pass kernels: storage c64, transform sign -1.
#define WSFFT_IO IoC64
#define WSFFT_SIGN (-1)
#define WSFFT_FIND find_pass_c64_neg
#define WSFFT_FIND_FUSED find_fused_c64_neg
#include "pass_inst.inc"
