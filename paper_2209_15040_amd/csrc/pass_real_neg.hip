// Real-data pencil-pass kernels: storage c64, transform sign -1.
#define WSFFT_IO IoC64
#define WSFFT_SIGN (-1)
#define WSFFT_REAL_ONLY
#define WSFFT_FIND_REAL find_real_c64_neg
#include "pass_inst.inc"
