// hc_distinct.hip -- duplicate marking of a set of points on the device: the
// merge step of monodromy (new endpoints of a loop joined to the known
// solutions; the paper computes its start systems offline by monodromy,
// section 7).
//
// keep[i] = 1 unless an earlier point j < i lies within the relative tolerance:
// max_k |x_ik - x_jk| <= tol max(s_i, s_j), s = max(1, |x|_inf).  One thread per
// point i; the points j < i are staged through LDS a tile at a time as a complex
// projection sum_k w_k x_jk (fixed generic weights) and their scale s_j.  Two
// points within the tolerance have projections within W tol max(s_i, s_j),
// W = sum_k |w_k| (each complex entry differs by at most tol max(s_i, s_j) in
// modulus); only those candidates are compared in full.
#include <cmath>

#include "hc_device.h"

namespace hcx {

namespace {

constexpr int kTile = 1024;

__device__ __forceinline__ cx<double> dweight(int k) { return {cos(0.7 * k + 0.3), sin(1.9 * k + 1.1)}; }

__device__ __forceinline__ void proj_scale(int n, const double *x, cx<double> &p, double &s)
{
    p = {0.0, 0.0};
    s = 1.0;
    for (int k = 0; k < n; k++) {
        const cx<double> v = {x[2 * k], x[2 * k + 1]};
        p = cfma(dweight(k), v, p);
        s = fmax(s, sqrt(abs2(v)));
    }
}

__global__ __launch_bounds__(256) void k_distinct(int n, long long count, const double *pts, double tol, double wsum,
                                                  int *keep)
{
    __shared__ cx<double> tp[kTile];
    __shared__ double ts[kTile];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool mine = i < count;
    cx<double> pi = {0.0, 0.0};
    double si = 1.0;
    if (mine) proj_scale(n, pts + (size_t)i * n * 2, pi, si);
    bool dup = !mine;
    // rows before this block's last row
    const long long last = min(count, (long long)(blockIdx.x + 1) * blockDim.x);
    for (long long j0 = 0; j0 < last; j0 += kTile) {
        const int m = (int)min((long long)kTile, last - j0);
        __syncthreads();
        for (int t = threadIdx.x; t < m; t += blockDim.x) {
            cx<double> p;
            double s;
            proj_scale(n, pts + (size_t)(j0 + t) * n * 2, p, s);
            tp[t] = p;
            ts[t] = s;
        }
        __syncthreads();
        for (int t = 0; !dup && t < m && j0 + t < i; t++) {
            const double lim = tol * fmax(si, ts[t]);
            if (sqrt(abs2(cx<double>{pi.re - tp[t].re, pi.im - tp[t].im})) > wsum * lim * (1.0 + 1e-6)) continue;
            const double *xi = pts + (size_t)i * n * 2, *xj = pts + (size_t)(j0 + t) * n * 2;
            double d = 0.0;
            for (int k = 0; k < n; k++)
                d = fmax(d, sqrt(abs2(cx<double>{xi[2 * k] - xj[2 * k], xi[2 * k + 1] - xj[2 * k + 1]})));
            dup = d <= lim;
        }
    }
    if (mine) keep[i] = dup ? 0 : 1;
}

}  // namespace

hipError_t launch_distinct(int n, long long count, const double *pts, double tol, int *keep, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    double w = 0.0;
    for (int k = 0; k < n; k++) w += std::hypot(std::cos(0.7 * k + 0.3), std::sin(1.9 * k + 1.1));
    hipLaunchKernelGGL(k_distinct, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, n, count, pts, tol,
                       w, keep);
    return hipGetLastError();
}

}  // namespace hcx
