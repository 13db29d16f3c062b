// hc_device.h -- device-side helpers shared by the gfx950 kernels: complex
// arithmetic on (re, im) pairs, constant-address-space table reads and
// wavefront-level primitives.
#pragma once

#include "hc_internal.h"

namespace hcx {

// ---------------------------------------------------------------- complex helpers

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> acc)
{
    return {fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}
// acc - a * b
template <typename R>
__device__ __forceinline__ cx<R> cfms(cx<R> a, cx<R> b, cx<R> acc)
{
    return {fma(-a.re, b.re, fma(a.im, b.im, acc.re)), fma(-a.re, b.im, fma(-a.im, b.re, acc.im))};
}
template <typename R>
__device__ __forceinline__ cx<R> cscale(R s, cx<R> a)
{
    return {s * a.re, s * a.im};
}
template <typename R>
__device__ __forceinline__ R abs1(cx<R> a)
{
    return fabs(a.re) + fabs(a.im);
}
template <typename R>
__device__ __forceinline__ R abs2(cx<R> a)
{
    return fma(a.re, a.re, a.im * a.im);
}

__device__ __forceinline__ double recip(double d) { return 1.0 / d; }
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }

template <typename R>
__device__ __forceinline__ cx<R> crecip(cx<R> a)
{
    R inv = recip(abs2(a));
    return {a.re * inv, -a.im * inv};
}

// Kernel tables are read-only for a whole launch.  Reading them through the
// constant address space lets the compiler use scalar loads (s_load into SGPRs)
// whenever the address is wavefront-uniform.
template <typename R>
using tbl_ptr = const __attribute__((address_space(4))) R *;

template <typename R>
__device__ __forceinline__ tbl_ptr<R> as_table(const R *p)
{
    return (tbl_ptr<R>)p;
}

template <typename R>
__device__ __forceinline__ cx<R> ldc(tbl_ptr<R> p, int k)
{
    return {p[2 * k], p[2 * k + 1]};
}

template <typename R>
__device__ __forceinline__ bool finite(cx<R> a)
{
    return isfinite(a.re) && isfinite(a.im);
}

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Blocks are dealt round-robin over the 8 XCDs; remapping them makes the blocks
// of one XCD take consecutive work items (same instance -> same L2 lines).
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    if (nb % 8 != 0) return b;
    return (b % 8) * (nb / 8) + b / 8;
}

}  // namespace hcx
