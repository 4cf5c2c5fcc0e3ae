// Peak microbenchmarks: the rates the rooflines divide by, measured on the
// device at hand (a streaming copy for HBM, back-to-back MFMA instructions
// of one kind for the matrix cores).

#include "kdev.hpp"
#include "kernels.hpp"

namespace ustat {
namespace {

constexpr int kPeakChains = 8;  // independent accumulator chains per wave

template <int KIND>
struct PeakOp;
template <>
struct PeakOp<0> {  // bf16 16x16x32, fp32 accumulation
    typedef f32x4 Acc;
    static constexpr double kFlops = 2.0 * 16 * 16 * 32;
    __device__ static Acc step(bf16x8 a, bf16x8 b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static bf16x8 operand(float v) {
        bf16x8 r;
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = (__bf16)(v + 0.125f * e);
        return r;
    }
};
template <>
struct PeakOp<1> {  // fp64 16x16x4
    typedef f64x4 Acc;
    static constexpr double kFlops = 2.0 * 16 * 16 * 4;
    __device__ static Acc step(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static double operand(float v) { return (double)v; }
};
template <>
struct PeakOp<2> {  // int8 16x16x64, int32 accumulation
    typedef i32x4 Acc;
    static constexpr double kFlops = 2.0 * 16 * 16 * 64;
    __device__ static Acc step(i32x4 a, i32x4 b, Acc c) {
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
    }
    __device__ static i32x4 operand(float v) {
        const int x = (int)v & 0x01010101;
        return i32x4{x, x, x, x};
    }
};
template <>
struct PeakOp<3> {  // fp32 16x16x4
    typedef f32x4 Acc;
    static constexpr double kFlops = 2.0 * 16 * 16 * 4;
    __device__ static Acc step(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static float operand(float v) { return v; }
};

// Every wave issues `iters` rounds of kPeakChains independent MFMAs on
// register operands formed from a run-time value (nothing folds); the sum of
// its accumulators goes to the sink so that none of the work is dead.
template <int KIND>
__global__ __launch_bounds__(256) void k_peak_mfma(float v, int64_t iters, char *sink) {
    typedef PeakOp<KIND> Op;
    typedef typename Op::Acc Acc;
    const int lane = threadIdx.x & 63;
    const auto a = Op::operand(v * (float)(lane + 1));
    const auto b = Op::operand(v * (float)(64 - lane));
    Acc acc[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = Acc{0, 0, 0, 0};
    for (int64_t it = 0; it < iters; ++it)
#pragma unroll
        for (int c = 0; c < kPeakChains; ++c) acc[c] = Op::step(a, b, acc[c]);
    Acc s = acc[0];
#pragma unroll
    for (int c = 1; c < kPeakChains; ++c) s += acc[c];
    // any lane's value will do: slots are reused modulo the sink's size
    reinterpret_cast<Acc *>(sink)[(blockIdx.x * 256 + threadIdx.x) % kPeakSinkSlots] = s;
}

// Streaming copy, four 16-byte loads in flight per thread.
__global__ __launch_bounds__(256) void k_peak_copy(const u32x4 *__restrict__ src,
                                                   u32x4 *__restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 x0 = src[i], x1 = src[i + stride], x2 = src[i + 2 * stride],
                    x3 = src[i + 3 * stride];
        dst[i] = x0;
        dst[i + stride] = x1;
        dst[i + 2 * stride] = x2;
        dst[i + 3 * stride] = x3;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

template <int KIND>
hipError_t run_mfma(int blocks, int64_t iters, char *sink, hipStream_t s, double *flops) {
    hipLaunchKernelGGL(k_peak_mfma<KIND>, dim3((unsigned)blocks), dim3(256), 0, s, 0.001f, iters,
                       sink);
    *flops = (double)blocks * 4.0 * (double)iters * kPeakChains * PeakOp<KIND>::kFlops;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_peak_mfma(int kind, int blocks, int64_t iters, char *sink, hipStream_t s,
                            double *flops) {
    switch (kind) {
        case 0: return run_mfma<0>(blocks, iters, sink, s, flops);
        case 1: return run_mfma<1>(blocks, iters, sink, s, flops);
        case 2: return run_mfma<2>(blocks, iters, sink, s, flops);
        case 3: return run_mfma<3>(blocks, iters, sink, s, flops);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_peak_copy(const void *src, void *dst, int64_t bytes, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_peak_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), bytes / 16);
    return hipGetLastError();
}

}  // namespace ustat
