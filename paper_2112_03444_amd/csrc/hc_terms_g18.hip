// hc_terms_g18.hip -- term-list tracker kernels of kind 4 (any degree <= 8, n <= 18, 32 lanes per
// path, an 18-row solver).
#include "hc_terms_impl.h"

HC_TERMS_INSTANTIATE(4)
