// hc_terms_g32.hip -- term-list tracker kernels of kind 6 (any degree <= 8, n <= 32, 32 lanes per
// path, a 32-row solver): every term-list system above 20 unknowns.
#include "hc_terms_impl.h"

HC_TERMS_INSTANTIATE(6)
