// hc_terms_g16.hip -- term-list tracker kernels of kind 1 (any degree <= 8, n <= 16, 16 lanes per path).
#include "hc_terms_impl.h"

HC_TERMS_INSTANTIATE(1)
