// hc_endgame.hip -- the power-series end-game for paths that do not reach a
// regular endpoint (Morgan, Sommese and Wampler, "A power series method for
// computing singular solutions to nonlinear analytic systems", Numer. Math. 63,
// 1992; the paper itself has no end-game).
//
// With s = 1 - t a path near t = 1 is a power series in sigma = s^(1/c), c >= 1
// its cycle number.  The host re-tracks the candidates (FP64, from their start
// points) to t = 1 - s0 and then to t_k = 1 - s0 beta^k, k = 1, 2, ...; after
// each of those launches k_eg_sample takes the candidates' sample k in
// projective coordinates y = (1, x) / (a . (1, x)) on a fixed patch (bounded at
// infinity, where y_0 -> 0), estimates c from how fast the last three samples
// approach each other, extrapolates y(0) by the quadratic in sigma through them,
// and stops a candidate once two successive estimates agree.  One thread per
// candidate: the end-game runs on the few paths that failed, compacted into a
// list, so its sampling kernels are launch- and latency-bound, not ALU-bound.
#include "hc_device.h"

namespace hcx {

namespace {

__device__ __forceinline__ double cabs_(cx<double> a) { return sqrt(abs2(a)); }

// max over j of |v_j|, NaN if any entry is NaN
__device__ __forceinline__ double nmax(double m, double a) { return (a <= m) ? m : a; }

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) { return cmul(a, crecip(b)); }

// Patch entry j (j = 0..n): exp(2 pi i frac((j + 1) phi)), phi = (sqrt 5 - 1) / 2.
__device__ __forceinline__ cx<double> patch(int j)
{
    const double phi = 0.5 * (sqrt(5.0) - 1.0);
    double f = (j + 1) * phi;
    f -= floor(f);
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);
    return {cs, sn};
}

__device__ __forceinline__ double *ring_at(const EgArgs &a, int slot, int i)
{
    return a.ring + ((size_t)slot * a.m + i) * (a.n + 1) * 2;
}

}  // namespace

__global__ __launch_bounds__(256) void k_eg_select(const EgArgs a)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.total) return;
    const int st = a.status[g];
    const double t = a.s.t[g];
    const bool zone = t >= 1.0 - a.s0;
    bool cand;
    if (a.mode == 2)
        cand = st != HC_T_NONFINITE && zone;
    else
        cand = st == HC_T_REFINE_FAILED || st == HC_T_SINGULAR ||
               ((st == HC_T_MIN_STEP || st == HC_T_MAX_STEPS) && zone);
    a.s.status[g] = cand ? kRetrack : kDone;
    if (cand) a.list[atomicAdd(a.count, 1u)] = (int)g;
}

__global__ __launch_bounds__(256) void k_eg_sample(const EgArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m) return;
    const long long g = a.list[i];
    const TrackState S = a.s;
    // still tracked and at this sample's t (not failed, not finished before)
    if (S.status[g] != kRunning || S.t[g] != a.t_k) return;
    const int n = a.n, n1 = a.n + 1;
    // the sample in projective coordinates on the patch
    cx<double> den = patch(0);
    for (int j = 0; j < n; j++) den = cfma(patch(j + 1), cx<double>{S.xr[j * a.total + g], S.xi[j * a.total + g]}, den);
    const cx<double> inv = crecip(den);
    double *yc = ring_at(a, a.k % 3, i);
    yc[0] = inv.re;
    yc[1] = inv.im;
    for (int j = 0; j < n; j++) {
        const cx<double> y = cmul(cx<double>{S.xr[j * a.total + g], S.xi[j * a.total + g]}, inv);
        yc[2 * (j + 1)] = y.re;
        yc[2 * (j + 1) + 1] = y.im;
    }
    if (a.k < 3) return;
    const double *ya = ring_at(a, (a.k - 2) % 3, i), *yb = ring_at(a, (a.k - 1) % 3, i);
    // decay of the differences of consecutive samples: |y_k - y_(k+1)| ~ s_k^(1/c)
    double d1 = 0.0, d2 = 0.0;
    for (int j = 0; j < n1; j++) {
        d1 = nmax(d1, cabs_(cx<double>{ya[2 * j] - yb[2 * j], ya[2 * j + 1] - yb[2 * j + 1]}));
        d2 = nmax(d2, cabs_(cx<double>{yb[2 * j] - yc[2 * j], yb[2 * j + 1] - yc[2 * j + 1]}));
    }
    int c = 1;
    double q = 0.0;
    bool still = d2 == 0.0;  // the path has stopped moving: y(0) = the last sample
    if (!still) {
        if (!(d2 < d1)) {  // not decaying (yet): no estimate this time
            a.have_prev[i] = 0;
            return;
        }
        const double cr = log(a.beta) / log(d2 / d1);
        c = (int)floor(cr + 0.5);
        c = c < 1 ? 1 : (c > a.max_cycle ? a.max_cycle : c);
        q = pow(a.beta, 1.0 / c);
    }
    // quadratic in sigma through the three samples (at sigma0, q sigma0, q^2 sigma0),
    // evaluated at sigma = 0, compared with the previous estimate
    double *ep = a.prev + (size_t)i * n1 * 2;
    const bool hp = a.have_prev[i] != 0;
    double dn = 0.0, en = 0.0;
    cx<double> E0 = {0.0, 0.0};
    for (int j = 0; j < n1; j++) {
        cx<double> E;
        if (still) {
            E = {yc[2 * j], yc[2 * j + 1]};
        } else {
            const cx<double> y0 = {ya[2 * j], ya[2 * j + 1]}, y1 = {yb[2 * j], yb[2 * j + 1]},
                             y2 = {yc[2 * j], yc[2 * j + 1]};
            const double r1 = 1.0 / (1.0 - q);
            const cx<double> ra = {(y1.re - q * y0.re) * r1, (y1.im - q * y0.im) * r1};
            const cx<double> rb = {(y2.re - q * y1.re) * r1, (y2.im - q * y1.im) * r1};
            const double r2 = 1.0 / (1.0 - q * q);
            E = {(rb.re - q * q * ra.re) * r2, (rb.im - q * q * ra.im) * r2};
        }
        if (j == 0) E0 = E;
        if (hp) dn = nmax(dn, cabs_(cx<double>{E.re - ep[2 * j], E.im - ep[2 * j + 1]}));
        en = nmax(en, cabs_(E));
        ep[2 * j] = E.re;
        ep[2 * j + 1] = E.im;
    }
    a.have_prev[i] = 1;
    if (!hp) return;
    // settled on a finite point, or on y_0 = 0 as closely as the affine bound
    // |x| <= inf_bound can tell (a path to infinity)
    if (!(dn <= a.tol * en || (dn <= a.tol_inf * en && cabs_(E0) * a.inf_bound <= en))) return;
    // the estimate in affine coordinates x = y_(1..n) / y_0 (now in prev)
    double big = 0.0;
    for (int j = 0; j < n; j++) {
        const cx<double> x = cdiv(cx<double>{ep[2 * (j + 1)], ep[2 * (j + 1) + 1]}, E0);
        S.xr[j * a.total + g] = x.re;
        S.xi[j * a.total + g] = x.im;
        big = nmax(big, cabs_(x));
    }
    S.succ[g] = c;  // the cycle number, read back by the refinement's info
    S.status[g] = kDone;
    if (!(big <= a.inf_bound)) {
        // a path to infinity: written out here
        a.cls[i] = 3;
        for (int j = 0; j < n; j++) {
            a.endpoints[(g * n + j) * 2] = S.xr[j * a.total + g];
            a.endpoints[(g * n + j) * 2 + 1] = S.xi[j * a.total + g];
        }
        a.status[g] = HC_T_AT_INFINITY;
        if (a.info) {
            hc_track_info inf;
            inf.steps = S.steps[g];
            inf.rejects = S.rejects[g];
            inf.newton_its = S.nits[g];
            inf.refine_its = 0;
            inf.escalated = S.escal[g] != 0 ? 1 : 0;
            inf.cycle = c;
            inf.residual = NAN;
            a.info[g] = inf;
        }
    } else {
        a.cls[i] = c == 1 ? 1 : 2;
    }
}

__global__ __launch_bounds__(256) void k_eg_mark(const EgArgs a, int cls)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m) return;
    a.s.status[a.list[i]] = a.cls[i] == cls ? kReached : kDone;
}

hipError_t launch_eg_select(const EgArgs &a, hipStream_t st)
{
    if (a.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eg_select, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_eg_sample(const EgArgs &a, hipStream_t st)
{
    if (a.m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eg_sample, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_eg_mark(const EgArgs &a, int cls, hipStream_t st)
{
    if (a.m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eg_mark, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, st, a, cls);
    return hipGetLastError();
}

}  // namespace hcx
