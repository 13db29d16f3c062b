// hc_terms_g20.hip -- term-list tracker kernels of kind 2 (any degree <= 8, n <= 20, 32 lanes per path).
#include "hc_terms_impl.h"

HC_TERMS_INSTANTIATE(2)
