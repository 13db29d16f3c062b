// hc_peak.hip -- measured vector FMA rate of the device, the denominator check
// of the trackers' ALU roofline.  Every lane runs independent FMA chains on
// register values (no memory traffic inside the timed loop), all operands in
// per-lane vector registers: an operand shared by the wavefront would sit in a
// scalar register, and that form issues markedly slower on gfx950 (65-74
// against 118-126 TFLOP/s for FP32).  Built like every other source here with
// packed FP32 switched off, so the FP32 figure is the rate of plain
// (one-lane-one-value) FP32 FMAs that the trackers' code runs on.
#include "hc_internal.h"

namespace hcx {

namespace {

constexpr int kChains = 32;        // independent accumulators per lane
constexpr int kPeakThreads = 256;  // per block

// acc <- acc * b + c, kChains chains per lane, `iters` rounds.  seed = {b, c,
// start, sentinel}; the sum of the accumulators is stored only if it equals the
// sentinel (never, for the seeds the launcher uses), which keeps the chains live.
template <typename R>
__global__ __launch_bounds__(kPeakThreads) void k_peak_fma(const R *__restrict__ seed, R *__restrict__ out,
                                                             int iters)
{
    // per-lane operands (vector registers); the perturbation keeps the chains
    // bounded (|b| < 1) and different in every lane
    const R b = seed[0] + R(threadIdx.x) * R(1e-9), c = seed[1] + R(threadIdx.x) * R(1e-9);
    R acc[kChains];
#pragma unroll
    for (int i = 0; i < kChains; i++) acc[i] = seed[2] + R(i) * R(1e-3) + R(threadIdx.x) * R(1e-6);
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int i = 0; i < kChains; i++) acc[i] = fma(acc[i], b, c);
    }
    R s = R(0);
#pragma unroll
    for (int i = 0; i < kChains; i++) s += acc[i];
    if (s == seed[3]) out[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

template <typename R>
hipError_t time_peak(int blocks, int iters, int reps, hipStream_t st, double *tflops)
{
    R *seed = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipMalloc(&seed, 4 * sizeof(R));
    if (err == hipSuccess) err = hipMalloc(&out, (size_t)blocks * kPeakThreads * sizeof(R));
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) {
        const R h[4] = {R(0.999), R(1e-3), R(0.5), R(-1)};
        err = hipMemcpyAsync(seed, h, sizeof h, hipMemcpyHostToDevice, st);
    }
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_peak_fma<R>, dim3(blocks), dim3(kPeakThreads), 0, st, seed, out, iters);  // warm-up
        err = hipEventRecord(e0, st);
    }
    for (int r = 0; err == hipSuccess && r < reps; r++) {
        hipLaunchKernelGGL(k_peak_fma<R>, dim3(blocks), dim3(kPeakThreads), 0, st, seed, out, iters);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess) {
        const double flop = 2.0 * kChains * (double)iters * blocks * kPeakThreads * reps;
        *tflops = ms > 0.0f ? flop / (ms * 1e-3) / 1e12 : 0.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (seed) (void)hipFree(seed);
    return err;
}

}  // namespace

hipError_t measure_peak_fma(bool fp64, double *tflops, hipStream_t st)
{
    int dev = 0, cus = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    // 8 blocks of 4 wavefronts per CU: 8 wavefronts per SIMD to hide the FMA latency
    const int blocks = 8 * (cus > 0 ? cus : 1);
    return fp64 ? time_peak<double>(blocks, 2048, 20, st, tflops) : time_peak<float>(blocks, 2048, 20, st, tflops);
}

}  // namespace hcx
