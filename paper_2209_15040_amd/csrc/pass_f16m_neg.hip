// Direct pencil-pass kernels: storage f16 with FP16 arithmetic, transform sign -1.
#define WSFFT_IO IoF16M
#define WSFFT_SIGN (-1)
#define WSFFT_FIND find_pass_f16m_neg
#include "pass_inst.inc"
