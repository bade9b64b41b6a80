// Contiguous passes with streaming loads and cached stores (BF16 storage, FP32 arithmetic,
// transform sign +1): the x pass of a plane chunk whose y pass follows at once.
#define WSFFT_IO IoBF16
#define WSFFT_SIGN 1
#define WSFFT_CACHE_ONLY
#define WSFFT_CACHE_STORE_ONLY
#define WSFFT_FIND_CACHE find_cached_bf16_pos
#include "pass_inst.inc"
