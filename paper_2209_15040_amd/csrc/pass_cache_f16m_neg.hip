// Contiguous passes with streaming loads and cached stores (FP16 storage and arithmetic,
// transform sign -1): the x pass of a plane chunk whose y pass follows at once.
#define WSFFT_IO IoF16M
#define WSFFT_SIGN (-1)
#define WSFFT_CACHE_ONLY
#define WSFFT_CACHE_STORE_ONLY
#define WSFFT_FIND_CACHE find_cached_f16m_neg
#include "pass_inst.inc"
