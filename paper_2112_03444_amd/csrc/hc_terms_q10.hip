// hc_terms_q10.hip -- term-list tracker kernels of kind 5 (degree <= 2, n <= 10, 16 lanes per path,
// a 10-row solver).
#include "hc_terms_impl.h"

HC_TERMS_INSTANTIATE(5)
