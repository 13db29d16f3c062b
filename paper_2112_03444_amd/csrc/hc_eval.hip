// hc_eval.hip -- batched FP32 evaluation of a dense quadratic system F and its
// Jacobian at many points of each instance (the evaluation step of section 3's
// tracker, Eq. (3)-(4), and section 6's parallel evaluation), by two engines:
//
//   rows:  one Jacobian row per lane, eight lanes per point, the coefficients
//          read from LDS -- the evaluation the group trackers run every stage;
//   mfma:  the same numbers as matrix products on the matrix cores.  With
//          y = (x, 1), row r of the Jacobian is M_r y for the n x (n + 1)
//          complex matrix M_r = [Q_r | L_r] (Q_r symmetric, its diagonal the
//          doubled square coefficients), so the n^2 x (n + 1) stack of all rows
//          times the points of one instance, [y_1 ... y_P], is one matrix
//          product per instance.  In real arithmetic it is the 2 n^2 x 2 (n + 1)
//          matrix [[Re M, -Im M], [Im M, Re M]] times the stacked real and
//          imaginary parts of the points, run as v_mfma_f32_16x16x4_f32 tiles:
//          16 points per wavefront, one tile of 16 rows per unknown a (the
//          pairs (equation r, re/im) of the entries J_r[a]), 2 (n + 1) rounded
//          up to a multiple of 4 in the reduction dimension.
//
// F_r follows from the row by Euler's identity for a quadratic:
// F_r = c_r + (L_r . x + x . (J_r x-row)) / 2 with J_r the row (L_r + Q_r x).
// `repeat` evaluates every point that many times (results of one evaluation);
// it exists to time the arithmetic apart from the memory traffic, since one
// evaluation of a point moves more bytes (8 n (n + 2) out) than its FLOPs keep
// the ALUs busy for.
#include "hc_device.h"

namespace hcx {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Empty compiler barriers of the timing loop: the point becomes opaque at the
// top of each evaluation (so nothing is hoisted out of the loop) and the
// results are consumed at its bottom (so nothing is dropped).
__device__ __forceinline__ void opaque(float &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void consume(float v) { asm volatile("" : : "v"(v)); }
__device__ __forceinline__ void consume(f32x4 v) { asm volatile("" : : "v"(v)); }
__device__ __forceinline__ void memory_barrier() { asm volatile("" : : : "memory"); }

constexpr int nterms(int n) { return 1 + n + n * (n + 1) / 2; }

// Table slot of the quadratic term x_a x_b (a <= b) in an equation's row:
// constant, n linear terms, then the pairs a <= b in row-major order.
__device__ __forceinline__ int pair_slot(int n, int a, int b)
{
    return 1 + n + a * n - a * (a - 1) / 2 + (b - a);
}

template <int N>
__global__ __launch_bounds__(256) void k_eval_rows(EvalArgs a)
{
    constexpr int T = nterms(N);
    __shared__ cx<float> tab[T * N];  // term q of equation r at q * N + r
    const int chunks = (a.n_pts + 31) / 32;
    const int inst = blockIdx.x / chunks, chunk = blockIdx.x % chunks;
    const float *src = a.tab + (size_t)inst * N * T * 2;
    for (int e = threadIdx.x; e < N * T; e += blockDim.x) {
        const int r = e / T, q = e % T;
        tab[q * N + r] = {src[2 * e], src[2 * e + 1]};
    }
    __syncthreads();
    const int r = threadIdx.x & 7;
    const int p = chunk * 32 + (threadIdx.x >> 3);
    if (r >= N || p >= a.n_pts) return;
    const size_t pt = (size_t)inst * a.n_pts + p;
    float xr[N], xi[N];
#pragma unroll
    for (int j = 0; j < N; j++) {
        xr[j] = a.x[(pt * N + j) * 2];
        xi[j] = a.x[(pt * N + j) * 2 + 1];
    }
    cx<float> row[N], F;
    for (int it = 0; it < a.repeat; it++) {
        memory_barrier();
        cx<float> x[N];
#pragma unroll
        for (int j = 0; j < N; j++) {
            opaque(xr[j]);
            opaque(xi[j]);
            x[j] = {xr[j], xi[j]};
        }
        cx<float> Lx = {0.f, 0.f};
#pragma unroll
        for (int j = 0; j < N; j++) {
            row[j] = tab[(1 + j) * N + r];
            Lx = cfma(row[j], x[j], Lx);
        }
        int q = 1 + N;
#pragma unroll
        for (int i = 0; i < N; i++) {
#pragma unroll
            for (int j = i; j < N; j++) {
                const cx<float> c = tab[(q++) * N + r];
                if (i == j) {
                    row[i] = cfma(c, x[j], row[i]);
                } else {
                    row[i] = cfma(c, x[j], row[i]);
                    row[j] = cfma(c, x[i], row[j]);
                }
            }
        }
        cx<float> s = Lx;
#pragma unroll
        for (int j = 0; j < N; j++) s = cfma(x[j], row[j], s);
        const cx<float> c0 = tab[r];
        F = {fmaf(0.5f, s.re, c0.re), fmaf(0.5f, s.im, c0.im)};
#pragma unroll
        for (int j = 0; j < N; j++) {
            consume(row[j].re);
            consume(row[j].im);
        }
        consume(F.re);
        consume(F.im);
    }
    float *jo = a.J + (pt * N + r) * N * 2;
#pragma unroll
    for (int j = 0; j < N; j++) {
        jo[2 * j] = row[j].re;
        jo[2 * j + 1] = row[j].im;
    }
    a.F[(pt * N + r) * 2] = F.re;
    a.F[(pt * N + r) * 2 + 1] = F.im;
}

template <int N>
__global__ __launch_bounds__(256) void k_eval_mfma(EvalArgs a)
{
    constexpr int T = nterms(N);
    constexpr int KS = (2 * (N + 1) + 3) / 4;  // reduction steps of 4
    // One tile per unknown a: its 16 rows are (equation r, re/im) of the
    // entries J_r[a], its columns the real and imaginary parts of y_b.  The
    // A fragments sit in the order the lanes read them (tile a, step s, lane l
    // holds A[l % 16][4 s + l / 16]).  A lane's results then cover two whole
    // Jacobian rows (equations 2 q, 2 q + 1 of its quarter q) of one point, so
    // F follows within the lane.
    __shared__ float frag[N * KS * 64];
    __shared__ cx<float> lin[N * (N + 1)];  // L_r at r (N + 1) + j, c_r at r (N + 1) + N
    const int chunks = (a.n_pts + 63) / 64;
    const int inst = blockIdx.x / chunks, chunk = blockIdx.x % chunks;
    const float *src = a.tab + (size_t)inst * N * T * 2;
    for (int e = threadIdx.x; e < N * KS * 64; e += blockDim.x) {
        const int l = e & 63, s = (e >> 6) % KS, ua = (e >> 6) / KS;
        const int i = l & 15, k = 4 * s + (l >> 4);
        const int r = i >> 1, part = i & 1, b = k >> 1, kpart = k & 1;
        float v = 0.f;
        if (r < N && b <= N) {
            const int q = b == N ? 1 + ua : pair_slot(N, min(ua, b), max(ua, b));
            const float mr = src[(r * T + q) * 2], mi = src[(r * T + q) * 2 + 1];
            v = part == 0 ? (kpart == 0 ? mr : -mi) : (kpart == 0 ? mi : mr);
        }
        frag[e] = v;
    }
    for (int e = threadIdx.x; e < N * (N + 1); e += blockDim.x) {
        const int r = e / (N + 1), j = e % (N + 1);
        const int q = j < N ? 1 + j : 0;
        lin[e] = {src[(r * T + q) * 2], src[(r * T + q) * 2 + 1]};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pj = lane & 15, qd = lane >> 4;  // the lane's point in the tile, its quarter
    const int p = chunk * 64 + wave * 16 + pj;
    const bool live = p < a.n_pts;
    const size_t pt = (size_t)inst * a.n_pts + (live ? p : 0);
    // B operand: step s takes the real (qd even) or imaginary part of y_{2s + qd/2}
    float bv[KS];
#pragma unroll
    for (int s = 0; s < KS; s++) {
        const int b = 2 * s + (qd >> 1), part = qd & 1;
        bv[s] = !live ? 0.f : b < N ? a.x[(pt * N + b) * 2 + part] : (b == N && part == 0 ? 1.f : 0.f);
    }
    float xr[N], xi[N];
#pragma unroll
    for (int j = 0; j < N; j++) {
        xr[j] = live ? a.x[(pt * N + j) * 2] : 0.f;
        xi[j] = live ? a.x[(pt * N + j) * 2 + 1] : 0.f;
    }
    const int r0 = 2 * qd, r1 = 2 * qd + 1;  // this lane's equations (rows of J)
    const int l0 = min(r0, N - 1), l1 = min(r1, N - 1);
    f32x4 acc[N];
    cx<float> F0, F1;
    for (int it = 0; it < a.repeat; it++) {
        memory_barrier();
#pragma unroll
        for (int s = 0; s < KS; s++) opaque(bv[s]);
#pragma unroll
        for (int u = 0; u < N; u++) {
            acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; s++)
                acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(frag[(u * KS + s) * 64 + lane], bv[s], acc[u], 0, 0,
                                                              0);
        }
        // Euler: s_r = L_r . x + x . J_r for the lane's two equations
        cx<float> s0 = {0.f, 0.f}, s1 = {0.f, 0.f};
#pragma unroll
        for (int u = 0; u < N; u++) {
            opaque(xr[u]);
            opaque(xi[u]);
            const cx<float> x = {xr[u], xi[u]};
            const cx<float> L0 = lin[l0 * (N + 1) + u], L1 = lin[l1 * (N + 1) + u];
            s0 = cfma(x, cx<float>{L0.re + acc[u][0], L0.im + acc[u][1]}, s0);
            s1 = cfma(x, cx<float>{L1.re + acc[u][2], L1.im + acc[u][3]}, s1);
        }
        const cx<float> c0 = lin[l0 * (N + 1) + N], c1 = lin[l1 * (N + 1) + N];
        F0 = {fmaf(0.5f, s0.re, c0.re), fmaf(0.5f, s0.im, c0.im)};
        F1 = {fmaf(0.5f, s1.re, c1.re), fmaf(0.5f, s1.im, c1.im)};
#pragma unroll
        for (int u = 0; u < N; u++) consume(acc[u]);
        consume(F0.re);
        consume(F0.im);
        consume(F1.re);
        consume(F1.im);
    }
    if (!live) return;
    if (r0 < N) {
        float *jo = a.J + (pt * N + r0) * N * 2;
#pragma unroll
        for (int u = 0; u < N; u++) {
            jo[2 * u] = acc[u][0];
            jo[2 * u + 1] = acc[u][1];
        }
        a.F[(pt * N + r0) * 2] = F0.re;
        a.F[(pt * N + r0) * 2 + 1] = F0.im;
    }
    if (r1 < N) {
        float *jo = a.J + (pt * N + r1) * N * 2;
#pragma unroll
        for (int u = 0; u < N; u++) {
            jo[2 * u] = acc[u][2];
            jo[2 * u + 1] = acc[u][3];
        }
        a.F[(pt * N + r1) * 2] = F1.re;
        a.F[(pt * N + r1) * 2 + 1] = F1.im;
    }
}

template <int N>
hipError_t launch_n(const EvalArgs &a, int engine, hipStream_t st)
{
    const long long chunks = engine == 0 ? ((long long)a.n_pts + 31) / 32 : ((long long)a.n_pts + 63) / 64;
    const long long blocks = chunks * a.n_inst;
    if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
    if (engine == 0)
        hipLaunchKernelGGL(k_eval_rows<N>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_eval_mfma<N>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const EvalArgs &a, int engine, hipStream_t st)
{
    if ((long long)a.n_inst * a.n_pts == 0) return hipSuccess;
    switch (a.n) {
    case 1: return launch_n<1>(a, engine, st);
    case 2: return launch_n<2>(a, engine, st);
    case 3: return launch_n<3>(a, engine, st);
    case 4: return launch_n<4>(a, engine, st);
    case 5: return launch_n<5>(a, engine, st);
    case 6: return launch_n<6>(a, engine, st);
    case 7: return launch_n<7>(a, engine, st);
    case 8: return launch_n<8>(a, engine, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hcx
