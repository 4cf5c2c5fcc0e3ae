// Device-side helpers shared by the kernel translation units: element
// loads by dtype, accumulation domains, problem lookup in grouped launches,
// bf16 rounding and the XCD-aware block remap.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace ustat {

typedef __int128 i128;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- helpers

template <int DOM>
struct Dom;
template <>
struct Dom<DOM_FP> {
    typedef double acc;    // per-element products and vector values
    typedef double wide;   // scalar sums
};
template <>
struct Dom<DOM_INT> {
    typedef long long acc;
    typedef i128 wide;
};

__device__ __forceinline__ double load_fp(const void *p, int32_t dt, int64_t i) {
    switch (dt) {
        case DT_F64: return static_cast<const double *>(p)[i];
        case DT_F32: return (double)static_cast<const float *>(p)[i];
        case DT_I8: return (double)static_cast<const int8_t *>(p)[i];
        default: return (double)static_cast<const long long *>(p)[i];
    }
}
__device__ __forceinline__ long long load_int(const void *p, int32_t dt, int64_t i) {
    switch (dt) {
        case DT_I8: return (long long)static_cast<const int8_t *>(p)[i];
        case DT_I64: return static_cast<const long long *>(p)[i];
        case DT_F32: return (long long)static_cast<const float *>(p)[i];
        default: return (long long)static_cast<const double *>(p)[i];
    }
}
template <int DOM>
__device__ __forceinline__ typename Dom<DOM>::acc load_elem(const void *p, int32_t dt, int64_t i);
template <>
__device__ __forceinline__ double load_elem<DOM_FP>(const void *p, int32_t dt, int64_t i) {
    return load_fp(p, dt, i);
}
template <>
__device__ __forceinline__ long long load_elem<DOM_INT>(const void *p, int32_t dt, int64_t i) {
    return load_int(p, dt, i);
}

// Vectors are double (DOM_FP) or int64 (DOM_INT).
template <int DOM>
__device__ __forceinline__ typename Dom<DOM>::acc load_vec(const void *p, int64_t i) {
    return static_cast<const typename Dom<DOM>::acc *>(p)[i];
}


// Call f(T()) with T the element type named by dtype, so that loops over a
// matrix compile once per element type with no per-element branch.
template <class F>
__device__ __forceinline__ void with_dtype(int32_t dt, F &&f) {
    switch (dt) {
        case DT_F64: f(double()); break;
        case DT_F32: f(float()); break;
        case DT_I8: f(int8_t()); break;
        default: f((long long)0); break;
    }
}

// Locate the problem owning flat block index b (descriptors sorted by
// tile_start, first one at 0).
template <class D>
__device__ __forceinline__ int find_problem(const D *d, int nprob, int64_t b) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile_start <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}

// Rows of one column strip handled by a block (and thus the number of
// partial rows left for the fixed-order reduction: ceil(n / strip)).

// Four consecutive elements p[i .. i+3] of a row as the accumulation type;
// `vec` selects one wide load (the caller guarantees alignment and that all
// four lie inside the row), otherwise elements at or beyond `lim` read 0.
template <class T, class A>
__device__ __forceinline__ void load4(const T *p, int64_t i, bool vec, int64_t col, int64_t lim,
                                      A (&x)[4]) {
    if (vec) {
        if constexpr (sizeof(T) == 4) {
            typedef T v4 __attribute__((ext_vector_type(4)));
            v4 q = *reinterpret_cast<const v4 *>(p + i);
            x[0] = (A)q[0]; x[1] = (A)q[1]; x[2] = (A)q[2]; x[3] = (A)q[3];
        } else if constexpr (sizeof(T) == 8) {
            typedef T v2 __attribute__((ext_vector_type(2)));
            v2 q0 = *reinterpret_cast<const v2 *>(p + i);
            v2 q1 = *reinterpret_cast<const v2 *>(p + i + 2);
            x[0] = (A)q0[0]; x[1] = (A)q0[1]; x[2] = (A)q1[0]; x[3] = (A)q1[1];
        } else {
            typedef T v4 __attribute__((ext_vector_type(4)));
            v4 q = *reinterpret_cast<const v4 *>(p + i);
            x[0] = (A)q[0]; x[1] = (A)q[1]; x[2] = (A)q[2]; x[3] = (A)q[3];
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = (col + j < lim) ? (A)p[i + j] : (A)0;
    }
}

// Grouped column reductions: the NM distinct matrices of a group are read
// once per element for all of its outputs.  Block = 256 columns (4 per
// thread, 64 threads across) x d.strip rows (4 row groups).  The products
// of each output's row vectors over the strip are formed once per block in
// LDS (0 for rows past the end, which masks them).  T is the element type
// of every matrix of the launch (void: mixed types, dispatched per load).
// Rows are clamped into range instead of branched on, and 16-byte vector
// loads through the global address space are used whenever the thread's 4
// columns are in range and every row pitch is a multiple of 4 elements.
template <typename T, typename A>
__device__ __forceinline__ void load_row4(const MatRef &m, int64_t v, int64_t w, int64_t n,
                                          bool vec, A (&x)[4]) {
    if constexpr (std::is_void<T>::value) {
        with_dtype(m.dtype, [&](auto tag) {
            typedef decltype(tag) U;
            load4<U, A>(static_cast<const U *>(m.p), v * m.ld + w, vec, w, n, x);
        });
    } else {
        const T *p = static_cast<const T *>(m.p) + v * m.ld + w;
        if (vec) {
            if constexpr (sizeof(T) == 4) {
                typedef T v4 __attribute__((ext_vector_type(4)));
                const v4 q = *(const __attribute__((address_space(1))) v4 *)(p);
                x[0] = (A)q[0]; x[1] = (A)q[1]; x[2] = (A)q[2]; x[3] = (A)q[3];
            } else {
                typedef T v2 __attribute__((ext_vector_type(2)));
                const v2 q0 = *(const __attribute__((address_space(1))) v2 *)(p);
                const v2 q1 = *(const __attribute__((address_space(1))) v2 *)(p + 2);
                x[0] = (A)q0[0]; x[1] = (A)q0[1]; x[2] = (A)q1[0]; x[3] = (A)q1[1];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = (w + j < n) ? (A)p[j] : (A)0;
        }
    }
}

// Flat block index -> logical tile index.  Consecutive workgroups are
// dispatched round-robin over the 8 XCDs; this gives each XCD a contiguous
// range of logical tiles so that neighbouring tiles share its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t G) {
    const int64_t per = G / 8, rem = G % 8, x = bid % 8, idx = bid / 8;
    return x * per + (x < rem ? x : rem) + idx;
}

// Running maximum of |entries| kept for the exact path's limb counts: the
// block's largest value (cross-lane exchange within each wave, then the
// waves' maxima through LDS) recorded with one device-scope atomic.  Such
// atomics on a single address execute one after another, so one per lane
// would cost far more than the kernel's own work.  Every thread of the
// block calls this once (it synchronises the block); threads without a
// value pass 0.
__device__ __forceinline__ void block_atomic_max(unsigned long long *p, unsigned long long v) {
    __shared__ unsigned long long wmax[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (int)((blockDim.x + 63) >> 6);
        for (int q = 1; q < nw; ++q) v = wmax[q] > v ? wmax[q] : v;
        atomicMax(p, v);
    }
}

// Launchers of the grouped row-mode and column-mode reductions for one
// (domain, element type) pair, defined in their own translation units.
template <int DOM, typename T>
hipError_t launch_rowred_dt(const ColDesc *d, int nprob, dim3 grid, int nm, int nout, hipStream_t s);
template <int DOM, typename T>
hipError_t launch_colred_dt(const ColDesc *d, int nprob, dim3 grid, int nm, int nout, hipStream_t s);

}  // namespace ustat
