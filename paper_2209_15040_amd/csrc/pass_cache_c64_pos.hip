// Complex64 passes through the caches, transform sign +1: cached loads and
// stores (both layouts) and contiguous passes with cached stores.
#define WSFFT_IO IoC64
#define WSFFT_SIGN 1
#define WSFFT_CACHE_ONLY
#define WSFFT_FIND_CACHE find_cached_c64_pos
#include "pass_inst.inc"
