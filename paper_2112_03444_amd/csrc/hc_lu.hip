// hc_lu.hip -- standalone batched complex linear solves (section 6, "Linear
// System Solver": one fused kernel factors the augmented matrix [A | b] with
// partial pivoting, which applies L^-1 to b on the way, and back-substitutes
// with the cached U).  One system per group of G lanes, one row per lane,
// G = 4, 8, 16 or 32 >= n, rows of 4, 8, 12, 16, 20, 24 or 32 entries; the
// group solver is the path trackers' (hc_group.h).
#include "hc_group.h"

namespace hcx {

namespace {

// Systems [batch] of size n <= N <= G: A row-major ([k][i][j]), b and x [k][i],
// complex of R interleaved.  Block of 4 wavefronts, 256 / G systems per block;
// the solver's rows hold N + 1 entries (columns n..N-1 zero).
template <int N, int G, typename R>
__global__ __launch_bounds__(256) void k_lu_solve(int n, long long batch, const R *__restrict__ A,
                                                   const R *__restrict__ b, R *__restrict__ x, int *__restrict__ info)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & (G - 1);
    const int base = lane - r;
    const long long k0 = ((long long)blockIdx.x * 256 + threadIdx.x) / G;  // this group's system
    const bool valid = k0 < batch;
    const long long k = valid ? k0 : 0;  // spare groups solve system 0 and write nothing
    const bool own = r < n;
    cx<R> row[N + 1];
    const R *Ar = A + ((size_t)k * n + (own ? r : 0)) * n * 2;
#pragma unroll
    for (int j = 0; j < N; j++) {
        row[j] = (own && j < n) ? cx<R>{Ar[2 * j], Ar[2 * j + 1]} : cx<R>{R(0), R(0)};
    }
    row[N] = own ? cx<R>{b[((size_t)k * n + r) * 2], b[((size_t)k * n + r) * 2 + 1]} : cx<R>{R(0), R(0)};
    cx<R> xr;
    R nd;
    const bool sing = group_solve<N, G, R>(row, r, base, xr, nd, n);
    if (!valid) return;
    if (own) {
        x[((size_t)k * n + r) * 2] = xr.re;
        x[((size_t)k * n + r) * 2 + 1] = xr.im;
    }
    if (info && r == 0) info[k] = sing ? 1 : 0;
}

template <int N, int G, typename R>
hipError_t launch_lu(int n, long long batch, const void *A, const void *b, void *x, int *info, hipStream_t st)
{
    const long long groups_per_block = 256 / G;
    const long long blocks = (batch + groups_per_block - 1) / groups_per_block;
    hipLaunchKernelGGL((k_lu_solve<N, G, R>), dim3((unsigned)blocks), dim3(256), 0, st, n, batch,
                       static_cast<const R *>(A), static_cast<const R *>(b), static_cast<R *>(x), info);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lu_solve(int n, long long batch, bool fp32, const void *A, const void *b, void *x, int *info,
                           hipStream_t st)
{
    if (batch == 0) return hipSuccess;
    // rows of the smallest listed length >= n, lanes per system the power of two >= it
    auto go = [&](auto tag) -> hipError_t {
        using R = decltype(tag);
        if (n <= 4) return launch_lu<4, 4, R>(n, batch, A, b, x, info, st);
        if (n <= 8) return launch_lu<8, 8, R>(n, batch, A, b, x, info, st);
        if (n <= 12) return launch_lu<12, 16, R>(n, batch, A, b, x, info, st);
        if (n <= 16) return launch_lu<16, 16, R>(n, batch, A, b, x, info, st);
        if (n <= 20) return launch_lu<20, 32, R>(n, batch, A, b, x, info, st);
        if (n <= 24) return launch_lu<24, 32, R>(n, batch, A, b, x, info, st);
        return launch_lu<32, 32, R>(n, batch, A, b, x, info, st);
    };
    return fp32 ? go(float()) : go(double());
}

}  // namespace hcx
