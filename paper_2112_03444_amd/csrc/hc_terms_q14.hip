// hc_terms_q14.hip -- term-list tracker kernels of kind 3 (degree <= 2, n <= 14, 16 lanes per path,
// a 14-row solver).
#include "hc_terms_impl.h"

HC_TERMS_INSTANTIATE(3)
