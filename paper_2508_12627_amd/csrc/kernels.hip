// HIP kernels for gfx950 (CDNA4): factor build, elimination steps, GEMMs
// on MFMA, fixed-order reductions and the Moebius combination.
//
// Every reduction is performed in a fixed order (per-tile partials written
// to memory, then summed in increasing tile index), so results are bitwise
// reproducible; no floating-point atomics are used anywhere.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <type_traits>

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

// ----------------------------------------------------------------- RBF

// RBF factor K(i,j) = exp(-||x_i - x_j||^2 / divisor) (Algorithm 1 with the
// kernel on an edge as the factor).  Only tiles on or above the diagonal
// are computed; each is written at (i, j) and, staged through LDS, at
// (j, i), so K is symmetric bit for bit and its diagonal is exactly 1.
// Squared distances are summed over coordinates in increasing order, in
// fp64, from direct differences.  Tile 64 x 64, each thread 4 x 4.
template <typename OT>
__device__ __forceinline__ void store4(OT *p, const double (&v)[4], bool vec, int64_t col,
                                       int64_t lim) {
    if (vec) {
        if constexpr (sizeof(OT) == 4) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            *reinterpret_cast<f4 *>(p) = f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        } else {
            typedef double d2 __attribute__((ext_vector_type(2)));
            reinterpret_cast<d2 *>(p)[0] = d2{v[0], v[1]};
            reinterpret_cast<d2 *>(p)[1] = d2{v[2], v[3]};
        }
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (col + c < lim) p[c] = (OT)v[c];
    }
}

template <typename OT>
__global__ __launch_bounds__(256) void k_rbf(const double *__restrict__ X, int64_t n, int32_t d,
                                             double inv_div, OT *__restrict__ out) {
    if (blockIdx.y > blockIdx.x) return;  // lower-triangle tiles come from the mirror
    __shared__ double sm[2 * 64 * 33];  // x rows of the tile's i and j ranges
    double(*xi)[33] = reinterpret_cast<double(*)[33]>(sm);
    double(*xj)[33] = reinterpret_cast<double(*)[33]>(sm + 64 * 33);
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    for (int k0 = 0; k0 < d; k0 += 32) {
        // clamped loads, all in flight together; entries outside the
        // samples or coordinates are zeroed afterwards
#pragma unroll
        for (int it = 0; it < 64 * 32 / 256; ++it) {
            const int e = t + 256 * it;
            const int rr = e >> 5, kk = e & 31;
            const int64_t gi = i0 + rr, gj = j0 + rr;
            const int gk = k0 + kk;
            const int gkc = min(gk, d - 1);
            const double a = X[min(gi, n - 1) * d + gkc];
            const double c = X[min(gj, n - 1) * d + gkc];
            xi[rr][kk] = (gi < n && gk < d) ? a : 0.0;
            xj[rr][kk] = (gj < n && gk < d) ? c : 0.0;
        }
        __syncthreads();
        const int kmax = min(32, d - k0);
        for (int kk = 0; kk < kmax; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = xi[ty * 4 + a][kk];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = xj[tx * 4 + c][kk];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double diff = av[a] - bv[c];
                    acc[a][c] = fma(diff, diff, acc[a][c]);
                }
        }
        __syncthreads();
    }
    double val[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) val[a][c] = exp(-acc[a][c] * inv_div);
    // direct tile: rows i0 + 4 ty + a, columns j0 + 4 tx + c (16-byte
    // stores when the row pitch keeps them aligned)
    const bool aligned = n % 4 == 0;
    {
        const int64_t j = j0 + tx * 4;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int64_t i = i0 + ty * 4 + a;
            if (i < n && j < n) store4<OT>(out + i * n + j, val[a], aligned && j + 3 < n, j, n);
        }
    }
    if (blockIdx.x == blockIdx.y) return;  // the diagonal tile is its own mirror
    // mirror tile: stage transposed in LDS, then write rows j0 + r, columns
    // i0 + 4 q .. i0 + 4 q + 3
    double *st = sm;  // 64 x 65 doubles
    static_assert(sizeof(sm) >= 64 * 65 * sizeof(double), "staging space");
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) st[(tx * 4 + c) * 65 + ty * 4 + a] = val[a][c];
    __syncthreads();
#pragma unroll
    for (int e = t; e < 64 * 16; e += 256) {
        const int r = e >> 4, q = e & 15;
        const int64_t j = j0 + r, i = i0 + 4 * q;
        if (j >= n || i >= n) continue;
        const double v4[4] = {st[r * 65 + 4 * q], st[r * 65 + 4 * q + 1], st[r * 65 + 4 * q + 2],
                              st[r * 65 + 4 * q + 3]};
        store4<OT>(out + j * n + i, v4, aligned && i + 3 < n, i, n);
    }
}

// ----------------------------------------------------------------- diag

template <int DOM>
__global__ void k_diag(const DiagDesc *__restrict__ D, int nprob) {
    const DiagDesc &d = D[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        typedef typename Dom<DOM>::acc A;
        A v = load_elem<DOM>(d.src.p, d.src.dtype, i * d.src.ld + i);
        static_cast<A *>(d.dst)[i] = v;
        if constexpr (DOM == DOM_INT) {
            if (d.mx_out) atomicMax(d.mx_out, (unsigned long long)(v < 0 ? -v : v));
        }
    }
}

// Largest |entry| of int8 matrices (one running max per problem).
__global__ void k_absmax_i8(const int8_t *const *src, const int64_t *n, int nprob,
                            unsigned long long *mx) {
    const int p = blockIdx.y;
    const int8_t *a = src[p];
    const int64_t cnt = n[p] * n[p];
    int best = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x) {
        int v = a[i];
        best = max(best, v < 0 ? -v : v);
    }
    __shared__ int red[256];
    red[threadIdx.x] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int q = 0; q < 256; ++q) m = max(m, red[q]);
        atomicMax(&mx[p], (unsigned long long)m);
    }
}

// ----------------------------------------------------------------- elim1

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

// Partials of y(w) = sum_v prod_k A_k(v,w) prod_j s_j(v) over a strip of
// 256 columns w and d.strip rows v.  Every operand is stored (v, w)
// (transposed operands arrive as materialised transposes), so each wave
// reads whole 1 KB row segments, four consecutive columns per lane.  Thread
// t owns columns w0 + 4 (t%64) .. +3 and rows v0 + t/64 + 4i of each 32-row
// chunk.
template <int DOM>
__global__ __launch_bounds__(256) void k_elim1(const Elim1Desc *__restrict__ D, int nprob) {
    typedef typename Dom<DOM>::acc A;
    __shared__ A red[4][256];
    const int64_t b = blockIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, b));  // uniform
    const Elim1Desc &d = D[p];
    const int64_t local = b - d.tile_start;
    const int64_t tv = local / d.tiles_w, tw = local % d.tiles_w;
    const int64_t n = d.n, w0 = tw * 256;
    const int t = threadIdx.x, cg = t & 63, g = t >> 6;
    const int64_t w = w0 + 4 * cg;
    const int64_t vbeg = tv * d.strip, vend = min(n, vbeg + d.strip);
    A sum[4] = {0, 0, 0, 0};
    for (int64_t v0 = vbeg; v0 < vend; v0 += 32) {
        A pr[8][4];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int64_t v = v0 + g + 4 * i;
            A sv = (v < vend) ? (A)1 : (A)0;
            if (v < vend)
                for (int j = 0; j < d.nS; ++j) sv *= load_vec<DOM>(d.s[j], v);
#pragma unroll
            for (int j = 0; j < 4; ++j) pr[i][j] = (w + j < n) ? sv : (A)0;
        }
        // Fast path: up to two operands of one element type have all their
        // loads of the chunk in flight before any multiply.
        int k0 = 0;
        if (d.nA >= 2 && d.A[0].dtype == d.A[1].dtype) {
            const MatRef m0 = d.A[0], m1 = d.A[1];
            with_dtype(m0.dtype, [&](auto tag) {
                typedef decltype(tag) T;
                const T *p0 = static_cast<const T *>(m0.p);
                const T *p1 = static_cast<const T *>(m1.p);
                const bool vec0 = (w + 3 < n) && (m0.ld % 4 == 0);
                const bool vec1 = (w + 3 < n) && (m1.ld % 4 == 0);
                A x0[8][4], x1[8][4];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    int64_t v = v0 + g + 4 * i;
                    if (v < vend) {
                        load4<T, A>(p0, v * m0.ld + w, vec0, w, n, x0[i]);
                        load4<T, A>(p1, v * m1.ld + w, vec1, w, n, x1[i]);
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) x0[i][j] = x1[i][j] = 0;
                    }
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const bool dg = v0 + g + 4 * i == w + j;
                        A a0 = (m0.zdiag && dg) ? (A)0 : x0[i][j];
                        A a1 = (m1.zdiag && dg) ? (A)0 : x1[i][j];
                        pr[i][j] *= a0 * a1;
                    }
            });
            k0 = 2;
        }
        for (int k = k0; k < d.nA; ++k) {
            const MatRef m = d.A[k];
            with_dtype(m.dtype, [&](auto tag) {
                typedef decltype(tag) T;
                const T *mp = static_cast<const T *>(m.p);
                const bool vec = (w + 3 < n) && (m.ld % 4 == 0);
                A x[8][4];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    int64_t v = v0 + g + 4 * i;
                    if (v < vend) load4<T, A>(mp, v * m.ld + w, vec, w, n, x[i]);
                    else x[i][0] = x[i][1] = x[i][2] = x[i][3] = 0;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        A xv = x[i][j];
                        if (m.zdiag && v0 + g + 4 * i == w + j) xv = 0;
                        pr[i][j] *= xv;
                    }
            });
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) sum[j] += pr[i][j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[g][4 * cg + j] = sum[j];
    __syncthreads();
    const int64_t wc = w0 + t;
    if (wc < n) {
        A tot = red[0][t] + red[1][t] + red[2][t] + red[3][t];
        static_cast<A *>(d.part)[tv * n + wc] = tot;
    }
}

// Transpose: out[b * n + a] = in[a * ld + b] for a, b < n (64 x 64 tiles
// through LDS, both sides coalesced).
__global__ __launch_bounds__(256) void k_transpose(const TransDesc *__restrict__ D, int nprob) {
    __shared__ long long tile[64][65];
    const int64_t b = blockIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, b));  // uniform
    const TransDesc &d = D[p];
    const int64_t local = b - d.tile_start;
    const int64_t ta = local / d.tiles, tb = local % d.tiles;
    const int64_t n = d.n, a0 = ta * 64, b0 = tb * 64;
    const int t = threadIdx.x;
    with_dtype(d.dtype, [&](auto tag) {
        typedef decltype(tag) T;
        const T *src = static_cast<const T *>(d.src);
        T *dst = static_cast<T *>(d.dst);
#pragma unroll 4
        for (int e = t; e < 4096; e += 256) {
            int r = e >> 6, c = e & 63;
            int64_t aa = a0 + r, bb = b0 + c;
            T v = (aa < n && bb < n) ? src[aa * d.ld + bb] : (T)0;
            tile[c][r] = (long long)0;
            *reinterpret_cast<T *>(&tile[c][r]) = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int e = t; e < 4096; e += 256) {
            int r = e >> 6, c = e & 63;  // output row b0 + r, column a0 + c
            int64_t bb = b0 + r, aa = a0 + c;
            if (aa < n && bb < n) dst[bb * n + aa] = *reinterpret_cast<const T *>(&tile[r][c]);
        }
    });
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

// Row mode (every matrix of the group symmetric): the sum over v of
// M[v][w] equals the sum along row w.  A block owns kRowBlock rows w and a
// segment of d.strip columns v (256, 512 or 1024); it forms each output's
// vector products over the segment once in LDS (lane-minor, so that the
// reads of a wave touch consecutive words).  Each wave then streams its
// rows one at a time, 16 columns per lane with the next row's loads in
// flight: every element is converted once, each output raises its whole
// row slice to its exponents in a uniform loop over unrolled multiplies,
// and the lanes are reduced in a fixed butterfly order.  A diagonal
// excluded by an output is subtracted once per row rather than masked per
// element.
template <int DOM, typename T, int NM, int NOUT>
__global__ __launch_bounds__(256) void k_rowred(const ColDesc *__restrict__ D, int nprob) {
    typedef typename Dom<DOM>::acc A;
    typedef typename std::conditional<std::is_void<T>::value, A, T>::type XT;
    constexpr int SEGMAX = 1024, RPW = kRowBlock / 4;
    __shared__ A svt[NOUT * SEGMAX];  // [output][q][j][lane]
    __shared__ A res[4][NOUT][RPW];   // reduced sums of each wave's rows
    const int64_t b = blockIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, b));  // uniform
    const ColDesc &d = D[p];
    const int64_t local = b - d.tile_start;
    const int64_t tr = local / d.tiles_v, ts = local % d.tiles_v;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t n = d.n;
    const int seg = d.strip, useg = seg / 256;
    const int64_t c0 = ts * seg;
    const int nout = d.nout;
    // matrix references and exponents, read once into uniform registers
    MatRef M[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) M[k] = d.M[k];
    int ex[NOUT][NM];
    bool zany[NOUT];  // the output excludes the diagonal
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        zany[o] = false;
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            ex[o][k] = __builtin_amdgcn_readfirstlane(o < nout ? (int)d.o[o].e[k] : 0);
            const bool z = __builtin_amdgcn_readfirstlane(o < nout ? (int)d.o[o].zd[k] : 0) != 0;
            zany[o] = zany[o] || (z && ex[o][k] > 0);
        }
    }
    // the segment's vector products: 0 past the end, past the segment and
    // for unused output slots
    {
        A sv[NOUT][SEGMAX / 256];
        int smax = 0;
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            if (o < nout) smax = max(smax, d.o[o].nS);
#pragma unroll
            for (int q = 0; q < SEGMAX / 256; ++q)
                sv[o][q] = (o < nout && q < useg && c0 + q * 256 + t < n) ? (A)1 : (A)0;
        }
        for (int jv = 0; jv < smax; ++jv)
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                if (o >= nout || jv >= d.o[o].nS) continue;
                const void *vp = d.o[o].s[jv];
#pragma unroll
                for (int q = 0; q < SEGMAX / 256; ++q) {
                    const int64_t v = min(c0 + q * 256 + t, n - 1);
                    sv[o][q] *= load_vec<DOM>(vp, v);
                }
            }
        const int sl = (t & 3) * 64 + (t >> 2);
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
            for (int q = 0; q < SEGMAX / 256; ++q) svt[o * SEGMAX + q * 256 + sl] = sv[o][q];
    }
    // whole 16-byte loads when every row pitch and n are multiples of 4
    // (uniform over the block)
    bool vecld = n % 4 == 0;
#pragma unroll
    for (int k = 0; k < NM; ++k) vecld = vecld && (M[k].ld % 4 == 0);
    __syncthreads();
    const int64_t wrow0 = tr * kRowBlock + wv * RPW;
    // Lane covers columns c0 + q * 256 + 4 * lane + j (element q * 4 + j of
    // its slice).  Loads have no branches: rows and columns are clamped
    // into range (clamped columns meet a zero vector product, rows past the
    // end are never stored).
    auto load_row = [&](XT (&x)[NM][16], int r, auto vec_tag) {
        constexpr bool VEC = decltype(vec_tag)::value;
        const int64_t w = min(wrow0 + r, n - 1);
#pragma unroll
        for (int k = 0; k < NM; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t v = c0 + q * 256 + 4 * lane;
                XT y[4];
                if constexpr (VEC) {
                    load_row4<T, XT>(M[k], w, min(v, n - 4), n, true, y);
#pragma unroll
                    for (int j = 0; j < 4; ++j) x[k][q * 4 + j] = y[j];
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        load_row4<T, XT>(M[k], w, min(v + j, n - 1), n, false, y);
                        x[k][q * 4 + j] = y[0];
                    }
                }
            }
    };
    auto run = [&](auto vec_tag) {
        // two register buffers used alternately (row indices are
        // compile-time constants after unrolling, so no copies)
        XT buf[2][NM][16];
        load_row(buf[0], 0, vec_tag);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            if (r + 1 < RPW) load_row(buf[(r + 1) & 1], r + 1, vec_tag);
            A xd[NM][16];
#pragma unroll
            for (int k = 0; k < NM; ++k)
#pragma unroll
                for (int e = 0; e < 16; ++e) xd[k][e] = (A)buf[r & 1][k][e];
            const int64_t w = wrow0 + r;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                if (o >= nout) break;
                A pr[16];
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    pr[e] = svt[o * SEGMAX + (e >> 2) * 256 + (e & 3) * 64 + lane];
#pragma unroll
                for (int k = 0; k < NM; ++k)
                    for (int c = 0; c < ex[o][k]; ++c)
#pragma unroll
                        for (int e = 0; e < 16; ++e) pr[e] *= xd[k][e];
                A acc = 0;
#pragma unroll
                for (int e = 0; e < 16; ++e) acc += pr[e];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
                // the diagonal term of an output that excludes it
                if (zany[o] && w < n && w >= c0 && w < c0 + seg) {
                    const int cw = (int)(w - c0);
                    A term = svt[o * SEGMAX + (cw >> 8) * 256 + (cw & 3) * 64 + ((cw & 255) >> 2)];
#pragma unroll
                    for (int k = 0; k < NM; ++k) {
                        XT y[4];
                        load_row4<T, XT>(M[k], w, w, n, false, y);
                        for (int c = 0; c < ex[o][k]; ++c) term *= (A)y[0];
                    }
                    acc -= term;
                }
                if (lane == 0) res[wv][o][r] = acc;
            }
        }
    };
    if (vecld) run(std::true_type{});
    else run(std::false_type{});
    __syncthreads();
    for (int idx = t; idx < 4 * NOUT * RPW; idx += 256) {
        const int w4 = idx / (NOUT * RPW), o = (idx / RPW) % NOUT, r = idx % RPW;
        const int64_t w = tr * kRowBlock + w4 * RPW + r;
        if (o < nout && w < n)
            ((__attribute__((address_space(1))) A *)(d.o[o].part))[ts * n + w] = res[w4][o][r];
    }
}

template <int DOM, typename T, int NM, int NOUT>
__global__ __launch_bounds__(256) void k_colred(const ColDesc *__restrict__ D, int nprob) {
    typedef typename Dom<DOM>::acc A;
    typedef typename std::conditional<std::is_void<T>::value, A, T>::type XT;
    constexpr int ROWS = 4;
    constexpr int CH = 4 * ROWS;  // rows per chunk of the block
    __shared__ A red[4][256];
    __shared__ A svt[NOUT * kElimStrip];  // [output][strip row]
    const int64_t b = blockIdx.x;
    // uniform over the block: descriptor fields become scalar loads
    const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, b));
    const ColDesc &d = D[p];
    const int64_t local = b - d.tile_start;
    const int64_t tv = local / d.tiles_w, tw = local % d.tiles_w;
    const int64_t n = d.n, w0 = tw * 256;
    const int t = threadIdx.x, cg = t & 63, g = t >> 6;
    const int64_t w = w0 + 4 * cg;
    const int strip = d.strip;
    const int64_t vbeg = tv * strip, vend = min(n, vbeg + strip);
    const int nout = d.nout;
    for (int idx = t; idx < NOUT * strip; idx += 256) {
        const int o = idx / strip, r = idx - o * strip;
        const int64_t v = vbeg + r;
        A sv = 0;  // rows past the end and unused output slots stay 0
        if (o < nout && v < vend) {
            sv = 1;
            for (int j = 0; j < d.o[o].nS; ++j) sv *= load_vec<DOM>(d.o[o].s[j], v);
        }
        svt[idx] = sv;
    }
    __syncthreads();
    bool vec = w + 3 < n;
#pragma unroll
    for (int k = 0; k < NM; ++k) vec = vec && (d.M[k].ld % 4 == 0);
    int ex[NOUT][NM];
    bool zd[NOUT][NM];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            ex[o][k] = o < nout ? d.o[o].e[k] : 0;
            zd[o][k] = o < nout && d.o[o].zd[k];
        }
    A sum[NOUT][4];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
        for (int j = 0; j < 4; ++j) sum[o][j] = 0;
    auto run = [&](auto vec_tag) {
        constexpr bool VEC = decltype(vec_tag)::value;
        for (int64_t v0 = vbeg; v0 < vend; v0 += CH) {
            XT x[NM][ROWS][4];
#pragma unroll
            for (int k = 0; k < NM; ++k)
#pragma unroll
                for (int i = 0; i < ROWS; ++i) {
                    const int64_t v = min(v0 + g + 4 * i, vend - 1);
                    load_row4<T, XT>(d.M[k], v, w, n, VEC, x[k][i]);
                }
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                const int64_t v = v0 + g + 4 * i;
                const int r = (int)min<int64_t>(v - vbeg, strip - 1);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool diag = v == w + j;
#pragma unroll
                    for (int o = 0; o < NOUT; ++o) {
                        if (o >= nout) break;
                        A pr = svt[o * strip + r];
#pragma unroll
                        for (int k = 0; k < NM; ++k) {
                            const A f = (zd[o][k] && diag) ? (A)0 : (A)x[k][i][j];
                            for (int e = 0; e < ex[o][k]; ++e) pr *= f;
                        }
                        sum[o][j] += (v < vend) ? pr : (A)0;
                    }
                }
            }
        }
    };
    if (vec) run(std::true_type{});
    else run(std::false_type{});
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        if (o >= nout) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) red[g][4 * cg + j] = (w + j < n) ? sum[o][j] : (A)0;
        __syncthreads();
        const int64_t wc = w0 + t;
        if (wc < n) {
            A tot = red[0][t] + red[1][t] + red[2][t] + red[3][t];
            static_cast<A *>(d.o[o].part)[tv * n + wc] = tot;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- reduce

// Non-dot: out[j] = prod mul(j) * sum_t part[t*stride + j] (vector domain
// type).  Dot: a single block sums those values over j into out[0] (wide
// type); `part` elements are wide when len == 1 (GEMM tile partials).
template <int DOM>
__global__ __launch_bounds__(256) void k_reduce(const ReduceDesc *__restrict__ D, int nprob) {
    typedef typename Dom<DOM>::acc A;
    typedef typename Dom<DOM>::wide Wd;
    const ReduceDesc &d = D[blockIdx.x];
    const int t = threadIdx.x;
    if (!d.dot) {
        // 64 columns per block pass; row group g sums partials q = g, g+4,
        // ... into two alternating accumulators, and the four groups are
        // combined in LDS, all in a fixed order
        __shared__ A cred[4][64];
        const int c = t & 63, g = t >> 6;
        const A *part = static_cast<const A *>(d.part);
        for (int64_t j0 = (int64_t)blockIdx.y * 64; j0 < d.len; j0 += (int64_t)gridDim.y * 64) {
            const int64_t j = j0 + c;
            A s0 = 0, s1 = 0;
            if (j < d.len) {
                int64_t q = g;
                for (; q + 4 < d.T; q += 8) {
                    s0 += part[q * d.stride + j];
                    s1 += part[(q + 4) * d.stride + j];
                }
                if (q < d.T) s0 += part[q * d.stride + j];
            }
            cred[g][c] = s0 + s1;
            __syncthreads();
            if (g == 0 && j < d.len) {
                A s = (cred[0][c] + cred[1][c]) + (cred[2][c] + cred[3][c]);
                for (int q = 0; q < d.nmul; ++q) s *= load_vec<DOM>(d.mul[q], j);
                static_cast<A *>(d.out)[j] = s;
                if constexpr (DOM == DOM_INT) {
                    if (d.mx_out) atomicMax(d.mx_out, (unsigned long long)(s < 0 ? -s : s));
                }
            }
            __syncthreads();
        }
        return;
    }
    if (blockIdx.y != 0) return;
    __shared__ Wd red[256];
    Wd acc = 0;
    if (d.len == 1) {
        // scalar (wide) partials: thread t sums q = t, t+256, ... in order
        for (int64_t q = t; q < d.T; q += 256) acc += static_cast<const Wd *>(d.part)[q * d.stride];
    } else {
        // four elements per thread per round (j, j + 256, ...), their loads
        // issued together from clamped indices; summed in that fixed order
        constexpr int U = 4;
        for (int64_t j0 = t; j0 < d.len; j0 += 256 * U) {
            A s[U];
#pragma unroll
            for (int u = 0; u < U; ++u) s[u] = 0;
            for (int64_t q = 0; q < d.T; ++q)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t j = min(j0 + 256 * u, d.len - 1);
                    s[u] += static_cast<const A *>(d.part)[q * d.stride + j];
                }
            Wd w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = (Wd)s[u];
            for (int q = 0; q < d.nmul; ++q)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    w[u] *= (Wd)load_vec<DOM>(d.mul[q], min(j0 + 256 * u, d.len - 1));
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j0 + 256 * u < d.len) acc += w[u];
        }
    }
    red[t] = acc;
    __syncthreads();
    // fixed-order tree
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
    if (t == 0) static_cast<Wd *>(d.out)[0] = red[0];
}

// ----------------------------------------------------------------- elim0

template <int DOM>
__global__ __launch_bounds__(256) void k_elim0(const Elim0Desc *__restrict__ D, int nprob) {
    typedef typename Dom<DOM>::wide Wd;
    __shared__ Wd red[256];
    const Elim0Desc &d = D[blockIdx.x];
    const int t = threadIdx.x;
    Wd acc = 0;
    // four elements per thread per round (v, v + 256, ...), their loads
    // issued together from clamped indices; summed in that fixed order
    constexpr int U = 4;
    for (int64_t v0 = t; v0 < d.n; v0 += 256 * U) {
        Wd x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = 1;
        for (int j = 0; j < d.nS; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] *= (Wd)load_vec<DOM>(d.s[j], min(v0 + 256 * u, d.n - 1));
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v0 + 256 * u < d.n) acc += x[u];
    }
    red[t] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
    if (t == 0) static_cast<Wd *>(d.out)[0] = red[0];
}

// ----------------------------------------------------------------- prep

// One 64 x 128 tile (rows w, columns v) of a GEMM operand
// out[w][v] = prod_j s_j(v) prod_k A_k(v, w) with every operand stored
// (w, v), so rows are read and written in order, four consecutive v per
// lane.  Thread t owns columns v0 + 4 (t%32) .. +3 and rows w0 + t/32 + 8i.
template <int DOM>
__global__ __launch_bounds__(256) void k_prep(const PrepDesc *__restrict__ D, int nprob) {
    typedef typename Dom<DOM>::acc A;
    const int64_t b = blockIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, b));  // uniform
    const PrepDesc &d = D[p];
    const int64_t local = b - d.tile_start;
    const int64_t tcol = d.npad / 128;
    const int64_t tw = local / tcol, tv = local % tcol;
    const int64_t n = d.n, w0 = tw * 64, v0 = tv * 128;
    const int t = threadIdx.x, cg = t & 31, rg = t >> 5;
    const int64_t v = v0 + 4 * cg;
    int limbs = d.limbs;
    if (d.format == PF_I8LIMBS) {
        // Digits needed for |x| <= prod of the operands' maxima: a top digit
        // in [-128, 127] above balanced digits in [-64, 63].
        double bound = 1.0;
        for (int q = 0; q < d.nmx; ++q) bound *= (double)*d.mx[q];
        int L = 1;
        double X = bound;
        while (X > 127.0 && L < d.limbs) {
            X = floor((X + 64.0) / 128.0);
            ++L;
        }
        limbs = L;
        if (local == 0 && t == 0) *d.limbs_out = L;
    }
    A sv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) sv[j] = (v + j < n) ? (A)1 : (A)0;
    for (int q = 0; q < d.nS; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) sv[j] *= load_vec<DOM>(d.s[q], min(v + j, n - 1));
    A pr[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int64_t w = w0 + rg + 8 * i;
#pragma unroll
        for (int j = 0; j < 4; ++j) pr[i][j] = (w < n) ? sv[j] : (A)0;
    }
    for (int k = 0; k < d.nA; ++k) {
        const MatRef m = d.A[k];
        with_dtype(m.dtype, [&](auto tag) {
            typedef decltype(tag) T;
            const T *mp = static_cast<const T *>(m.p);
            // Rows and columns are clamped into range instead of branched
            // on (pr is already 0 outside it), so the eight rows' loads are
            // in flight together; 16-byte loads when n and the row pitch
            // are multiples of 4 (uniform over the block).
            A x[8][4];
            if (n % 4 == 0 && m.ld % 4 == 0) {
                const int64_t vc = min(v, n - 4);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int64_t w = min(w0 + rg + 8 * i, n - 1);
                    load4<T, A>(mp, w * m.ld + vc, true, vc, n, x[i]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int64_t w = min(w0 + rg + 8 * i, n - 1);
#pragma unroll
                    for (int j = 0; j < 4; ++j) x[i][j] = (A)mp[w * m.ld + min(v + j, n - 1)];
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    A xv = x[i][j];
                    if (m.zdiag && w0 + rg + 8 * i == v + j) xv = 0;
                    pr[i][j] *= xv;
                }
        });
    }
    // output fields read once (the stores below would otherwise force
    // their reloads, each waiting for every store in flight)
    const int64_t npad = d.npad, ldo = d.ldo, plane = d.plane;
    void *const out = d.out;
    const int format = d.format;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int64_t w = w0 + rg + 8 * i;
        if (w >= npad) continue;
        int64_t o = w * ldo + v;
        switch (format) {
            case PF_F64: {
                typedef double v2 __attribute__((ext_vector_type(2)));
                *reinterpret_cast<v2 *>(static_cast<double *>(out) + o) = v2{(double)pr[i][0], (double)pr[i][1]};
                *reinterpret_cast<v2 *>(static_cast<double *>(out) + o + 2) = v2{(double)pr[i][2], (double)pr[i][3]};
                break;
            }
            case PF_F32: {
                *reinterpret_cast<f32x4 *>(static_cast<float *>(out) + o) =
                    f32x4{(float)pr[i][0], (float)pr[i][1], (float)pr[i][2], (float)pr[i][3]};
                break;
            }
            case PF_BF16X2: {
                typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
                u16x4 hi, lo;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    double xd = (double)pr[i][j];
                    uint16_t h = f32_to_bf16_rne((float)xd);
                    hi[j] = h;
                    lo[j] = f32_to_bf16_rne((float)(xd - (double)bf16_to_f32(h)));
                }
                *reinterpret_cast<u16x4 *>(static_cast<uint16_t *>(out) + o) = hi;
                *reinterpret_cast<u16x4 *>(static_cast<uint16_t *>(out) + o + plane) = lo;
                break;
            }
            default: {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    long long xi = (long long)pr[i][j];
                    for (int l = 0; l + 1 < limbs; ++l) {
                        long long md = ((xi % 128) + 128 + 64) % 128 - 64;  // balanced digit
                        static_cast<int8_t *>(out)[o + j + l * plane] = (int8_t)md;
                        xi = (xi - md) / 128;
                    }
                    static_cast<int8_t *>(out)[o + j + (int64_t)(limbs - 1) * plane] = (int8_t)xi;
                }
                break;
            }
        }
    }
}

// ----------------------------------------------------------------- GEMM
//
// Block tile 128 x 128, four waves in a 2 x 2 arrangement, each wave a
// 64 x 64 region of 4 x 4 MFMA blocks of 16 x 16.  Operands live in LDS as
// [row][k] with padding; every 16x16 MFMA family used here (f64 16x16x4,
// f32 16x16x4, bf16 16x16x32, i8 16x16x64) reads lane l's A fragment from
// row l%16 and B fragment from column l%16 at k-slot group l/16.  Result
// item r of lane l sits in column l%16 and row 4*(l/16)+r, except for the
// f64 instruction, whose rows are interleaved: row l/16 + 4*r.

template <int PREC>
struct GemmCfg;
template <>
struct GemmCfg<0> {  // fp64
    typedef double E;
    static constexpr int BK = 16, PLANES = 1;
};
template <>
struct GemmCfg<1> {  // fp32
    typedef float E;
    static constexpr int BK = 16, PLANES = 1;
};
template <>
struct GemmCfg<2> {  // bf16 hi/lo
    typedef uint16_t E;
    static constexpr int BK = 32, PLANES = 2;
};
template <>
struct GemmCfg<3> {  // int8 limb (one plane per pass)
    typedef int8_t E;
    static constexpr int BK = 64, PLANES = 1;
};

// Row within a 16x16 MFMA result block of item r held by `lane`.
template <int PREC>
__device__ __forceinline__ int mfma_row(int lane, int r) {
    if constexpr (PREC == 0) return (lane >> 4) + 4 * r;
    else return 4 * (lane >> 4) + r;
}

template <int PREC>
struct AccT {
    typedef f32x4 T;
};
template <>
struct AccT<0> {
    typedef f64x4 T;
};
template <>
struct AccT<3> {
    typedef i32x4 T;
};

// Block-tile shapes.  S128: 128 x 128, four waves (2 x 2) of 64 x 64.
// S256: 256 x 256, eight waves (2 x 4) of 128 x 64; it halves the operand
// re-reads per flop, for large problems whose tile count still fills the
// chip (fp32 and split-bf16 accumulators only: 128 registers per lane).
struct S128 {
    static constexpr int BM = 128, BN = 128, WN = 2, NT = 256, FM = 4, FN = 4;
};
struct S256 {
    static constexpr int BM = 256, BN = 256, WN = 4, NT = 512, FM = 8, FN = 4;
};

// Global <-> LDS staging of one R x BK tile (all planes) of an operand by
// NT threads.  fp64 rows are padded to 144 bytes.  The 64-byte rows of the
// other formats are XOR-swizzled in 16-byte chunks, chunk ^ s(row) with
// s(row) = ((row >> 1) & 3) ^ ((row >> 3) & 1): a 16-byte fragment read by
// lanes on consecutive rows then touches distinct banks whether the LDS
// serves 8 lanes over 32 banks or 16 lanes over 64 banks per cycle.
template <int PREC, int R, int NT>
struct TileIO {
    typedef GemmCfg<PREC> C;
    static constexpr int ROWB = C::BK * (int)sizeof(typename C::E);  // bytes per row
    static constexpr int UPR = ROWB / 16;                            // 16B units per row
    static constexpr int UNITS = R * UPR * C::PLANES;
    static constexpr int PER = UNITS / NT;
    static_assert(UNITS % NT == 0, "tile units must divide over the threads");
    static constexpr int LROW = (PREC == 0) ? ROWB + 16 : ROWB;
    static constexpr int PLANEB = R * LROW;
    static constexpr int STAGE = PLANEB * C::PLANES;

    __device__ static __forceinline__ int off(int row, int chunk) {
        if constexpr (PREC == 0) return row * LROW + chunk * 16;
        else return row * LROW + ((chunk ^ ((row >> 1) & 3) ^ ((row >> 3) & 1)) << 4);
    }
    __device__ static void load(u32x4 (&r)[PER], const char *base, int64_t ldb, int64_t planeb,
                                int64_t row0, int64_t k0b) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int u = threadIdx.x + NT * i;
            int pl = u / (R * UPR);
            int uu = u % (R * UPR);
            int row = uu / UPR, cu = uu % UPR;
            const char *g = base + (uint32_t)(pl * planeb + (row0 + row) * ldb + k0b + cu * 16);
            // a 32-bit offset from the uniform base (every operand buffer is
            // below 4 GiB, checked when the schedule is built); global address space:
            // these loads only count against vmcnt, so waiting for LDS
            // fragment reads never waits for the prefetch
            r[i] = *(const __attribute__((address_space(1))) u32x4 *)(g);
        }
    }
    __device__ static void store(const u32x4 (&r)[PER], char *lds) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int u = threadIdx.x + NT * i;
            int pl = u / (R * UPR);
            int uu = u % (R * UPR);
            int row = uu / UPR, cu = uu % UPR;
            *reinterpret_cast<u32x4 *>(lds + pl * PLANEB + off(row, cu)) = r[i];
        }
    }
};

// One BK step of a wave's FM x FN blocks: A rows from ra0, B rows from rb0
// (tile-local), fragments read from LDS with the staging layout of R-row
// tiles (the layout does not depend on R).
template <int PREC, int FM, int FN, int RA, int RB>
__device__ __forceinline__ void mma_tile(typename AccT<PREC>::T (&acc)[FM][FN], const char *As,
                                         const char *Bs, int ra0, int rb0, int lane) {
    typedef TileIO<PREC, RA, 64> IOA;
    typedef TileIO<PREC, RB, 64> IOB;
    const int lr = lane & 15, lg = lane >> 4;
    if constexpr (PREC == 0) {
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            double a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = *reinterpret_cast<const double *>(As + (ra0 + i * 16 + lr) * IOA::LROW +
                                                         (kk + lg) * 8);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[j] = *reinterpret_cast<const double *>(Bs + (rb0 + j * 16 + lr) * IOB::LROW +
                                                         (kk + lg) * 8);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    } else if constexpr (PREC == 1) {
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            float a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = *reinterpret_cast<const float *>(As + IOA::off(ra0 + i * 16 + lr, kk >> 2) +
                                                        lg * 4);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[j] = *reinterpret_cast<const float *>(Bs + IOB::off(rb0 + j * 16 + lr, kk >> 2) +
                                                        lg * 4);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    } else if constexpr (PREC == 2) {
        bf16x8 bh[FN], bl[FN];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int rb = IOB::off(rb0 + j * 16 + lr, lg);
            bh[j] = *reinterpret_cast<const bf16x8 *>(Bs + rb);
            bl[j] = *reinterpret_cast<const bf16x8 *>(Bs + IOB::PLANEB + rb);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const int ra = IOA::off(ra0 + i * 16 + lr, lg);
            const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(As + ra);
            const bf16x8 al = *reinterpret_cast<const bf16x8 *>(As + IOA::PLANEB + ra);
            // small cross terms first, then the leading hi*hi term
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
            }
        }
    } else {
        i32x4 a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
            a[i] = *reinterpret_cast<const i32x4 *>(As + IOA::off(ra0 + i * 16 + lr, lg));
#pragma unroll
        for (int j = 0; j < FN; ++j)
            b[j] = *reinterpret_cast<const i32x4 *>(Bs + IOB::off(rb0 + j * 16 + lr, lg));
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// LDS bytes of one double-buffered (A, B) stage pair for a shape.
template <int PREC, class SH>
constexpr int gemm_stage_bytes() {
    return TileIO<PREC, SH::BM, SH::NT>::STAGE + TileIO<PREC, SH::BN, SH::NT>::STAGE;
}

// K loop of one (A plane set, B plane set) pass with register prefetch and
// double-buffered LDS (one barrier per K step).
template <int PREC, class SH>
__device__ __forceinline__ void gemm_pass(typename AccT<PREC>::T (&acc)[SH::FM][SH::FN],
                                          const char *Ab, const char *Bb, int64_t ldb,
                                          int64_t planeb, int64_t w0, int64_t x0, int64_t npad,
                                          char *lds) {
    typedef TileIO<PREC, SH::BM, SH::NT> IOA;
    typedef TileIO<PREC, SH::BN, SH::NT> IOB;
    constexpr int PAIR = IOA::STAGE + IOB::STAGE;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ra0 = (wv / SH::WN) * SH::FM * 16, rb0 = (wv % SH::WN) * SH::FN * 16;
    constexpr int KB = GemmCfg<PREC>::BK * (int)sizeof(typename GemmCfg<PREC>::E);
    const int64_t nk = npad / GemmCfg<PREC>::BK;
    u32x4 ra[IOA::PER], rb[IOB::PER];
    IOA::load(ra, Ab, ldb, planeb, w0, 0);
    IOB::load(rb, Bb, ldb, planeb, x0, 0);
    IOA::store(ra, lds);
    IOB::store(rb, lds + IOA::STAGE);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        char *As = lds + cur * PAIR;
        char *Bs = As + IOA::STAGE;
        // Prefetch the next K tile (the last step re-reads its own tile into
        // the idle buffer, which keeps the loop free of branches).
        const int64_t kn = (kt + 1 < nk) ? kt + 1 : kt;
        IOA::load(ra, Ab, ldb, planeb, w0, kn * KB);
        IOB::load(rb, Bb, ldb, planeb, x0, kn * KB);
        // Keep the prefetch at the top of the step and its staging after
        // the MFMAs: left to itself the scheduler sinks the loads below the
        // MFMAs (or waits for them in the middle), exposing their latency.
        // fp64 and int8 keep the free schedule (their register budget is
        // already full).
        if constexpr (PREC == 1 || PREC == 2) __builtin_amdgcn_sched_barrier(0);
        mma_tile<PREC, SH::FM, SH::FN, SH::BM, SH::BN>(acc, As, Bs, ra0, rb0, lane);
        if constexpr (PREC == 1 || PREC == 2) __builtin_amdgcn_sched_barrier(0);
        char *An = lds + (1 - cur) * PAIR;
        IOA::store(ra, An);
        IOB::store(rb, An + IOA::STAGE);
        __syncthreads();
    }
}

// Flat block index -> logical tile index.  Consecutive workgroups are
// dispatched round-robin over the 8 XCDs; this gives each XCD a contiguous
// range of logical tiles so that neighbouring tiles share its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t G) {
    const int64_t per = G / 8, rem = G % 8, x = bid % 8, idx = bid / 8;
    return x * per + (x < rem ? x : rem) + idx;
}

template <int PREC, class SH>
__global__ __launch_bounds__(SH::NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_gemm(const GemmDesc *__restrict__ D, int nprob) {
    typedef typename AccT<PREC>::T AT;
    constexpr int FM = SH::FM, FN = SH::FN;
    static_assert(PREC == 1 || PREC == 2 || SH::BM == 128, "large tiles: fp32 accumulators only");
    extern __shared__ __align__(16) char lds[];
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, b));  // uniform
    const GemmDesc &d = D[p];
    const int64_t local = b - d.tile_start;
    // grouped tile order: 8 tile-rows per group, column-major inside it
    const int64_t T = d.tiles, GM = 8;
    const int64_t first = (local / (GM * T)) * GM;
    const int64_t gsz = (T - first) < GM ? (T - first) : GM;
    const int64_t lg = local - first * T;
    const int64_t tm = first + lg % gsz, tn = lg / gsz;
    const int64_t w0 = tm * SH::BM, x0 = tn * SH::BN;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wr0 = w0 + (wv / SH::WN) * FM * 16, xc0 = x0 + (wv % SH::WN) * FN * 16;
    constexpr int ES = (int)sizeof(typename GemmCfg<PREC>::E);
    const int64_t ldb = d.ld * ES, planeb = d.plane * ES;

    AT acc[FM][FN];
    long long resi[PREC == 3 ? FM : 1][PREC == 3 ? FN : 1][4];
    (void)resi;
    if constexpr (PREC == 3) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) resi[i][j][r] = 0;
        const int nla = d.la_p ? *d.la_p : d.la, nlb = d.lb_p ? *d.lb_p : d.lb;
        for (int la = 0; la < nla; ++la)
            for (int lb = 0; lb < nlb; ++lb) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = AT{0, 0, 0, 0};
                gemm_pass<PREC, SH>(acc, static_cast<const char *>(d.A) + la * planeb,
                                    static_cast<const char *>(d.B) + lb * planeb, ldb, planeb, w0,
                                    x0, d.npad, lds);
                const long long wgt = 1ll << (7 * (la + lb));
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) resi[i][j][r] += wgt * (long long)acc[i][j][r];
            }
    } else {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = AT{0, 0, 0, 0};
        gemm_pass<PREC, SH>(acc, static_cast<const char *>(d.A), static_cast<const char *>(d.B),
                            ldb, planeb, w0, x0, d.npad, lds);
    }
    // value(i, j, r) of row wr0+i*16+mfma_row(lane,r), column xc0+j*16+lane%16
    auto value = [&](int i, int j, int r) {
        if constexpr (PREC == 3) return resi[i][j][r];
        else return (double)acc[i][j][r];
    };

    const int64_t n = d.n;
    if (!d.final_) {
        if constexpr (PREC == 3) {
            if (d.mx_out) {
                unsigned long long mloc = 0;
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            long long v = resi[i][j][r];
                            unsigned long long a = (unsigned long long)(v < 0 ? -v : v);
                            mloc = a > mloc ? a : mloc;
                        }
                atomicMax(d.mx_out, mloc);
            }
        }
        // output fields read once: a reload after each store would wait for
        // every store in flight
        void *const C = d.C;
        const int64_t ldc = d.ldc;
        const bool c64 = d.dtype_c == DT_F64;
#pragma clang loop unroll(full)
        for (int ib = 0; ib < FM; ib += 4)
#pragma unroll
        for (int i = ib; i < ib + 4; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int64_t w = wr0 + i * 16 + mfma_row<PREC>(lane, r);
                    int64_t x = xc0 + j * 16 + (lane & 15);
                    if (w < n && x < n) {
                        int64_t o = w * ldc + x;
                        if constexpr (PREC == 3) static_cast<long long *>(C)[o] = value(i, j, r);
                        else if (c64) static_cast<double *>(C)[o] = value(i, j, r);
                        else static_cast<float *>(C)[o] = (float)value(i, j, r);
                    }
                }
        return;
    }
    // Fused consumer: sum_{w,x} C(w,x) prod Z(w,x) prod aw(w) prod bx(x).
    typedef typename std::conditional<PREC == 3, i128, double>::type Wd;
    Wd part = 0;
#pragma clang loop unroll(full)
    for (int ib = 0; ib < FM; ib += 4)
#pragma unroll
    for (int i = ib; i < ib + 4; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t w = wr0 + i * 16 + mfma_row<PREC>(lane, r);
                int64_t x = xc0 + j * 16 + (lane & 15);
                if (w >= n || x >= n) continue;
                Wd val = (Wd)value(i, j, r);
                for (int k = 0; k < d.nZ; ++k) {
                    const MatRef &z = d.Z[k];
                    int64_t idx = z.trans ? (x * z.ld + w) : (w * z.ld + x);
                    Wd zv;
                    if constexpr (PREC == 3) zv = (Wd)load_int(z.p, z.dtype, idx);
                    else zv = load_fp(z.p, z.dtype, idx);
                    if (z.zdiag && w == x) zv = 0;
                    val *= zv;
                }
                for (int q = 0; q < d.naw; ++q) {
                    if constexpr (PREC == 3) val *= (Wd) static_cast<const long long *>(d.aw[q])[w];
                    else val *= static_cast<const double *>(d.aw[q])[w];
                }
                for (int q = 0; q < d.nbx; ++q) {
                    if constexpr (PREC == 3) val *= (Wd) static_cast<const long long *>(d.bx[q])[x];
                    else val *= static_cast<const double *>(d.bx[q])[x];
                }
                part += val;
            }
    __syncthreads();  // LDS reuse
    Wd *red = reinterpret_cast<Wd *>(lds);
    red[threadIdx.x] = part;
    __syncthreads();
    // fixed-order tree over the NT partial sums
    for (int s = SH::NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) static_cast<Wd *>(d.part)[local] = red[0];
}

// ----------------------------------------------------------------- combine

// One block per dataset: thread t forms V_p and mu_p * a_p of program
// p = p0 + t (the chains of index and scalar loads of different programs
// overlap), then thread 0 adds the terms to U and S in program order, the
// same order as a serial loop.
template <int DOM>
__global__ __launch_bounds__(256) void k_combine(
    const CombineDesc *__restrict__ D, int ndata, const int32_t *__restrict__ term_off,
    const int32_t *__restrict__ term_cnt, const int32_t *__restrict__ off,
    const int32_t *__restrict__ cnt, const int32_t *__restrict__ idx,
    const int64_t *__restrict__ mu, const void *__restrict__ scal, void *__restrict__ accv,
    int first, int last, void *__restrict__ uout, double *__restrict__ sout) {
    typedef typename Dom<DOM>::wide Wd;
    __shared__ Wd tvs[256];
    const int ds = blockIdx.x, t = threadIdx.x;
    if (ds >= ndata) return;
    const Wd *sc = static_cast<const Wd *>(scal);
    Wd *acc = static_cast<Wd *>(accv);
    const int pb = D[ds].p_begin, pe = D[ds].p_end;
    Wd U = 0;
    double S = 0;
    for (int p0 = pb; p0 < pe; p0 += 256) {
        const int p = p0 + t;
        Wd tv = 0;
        if (p < pe) {
            Wd V = 0;
            for (int k = term_off[p]; k < term_off[p] + term_cnt[p]; ++k) {
                Wd prod = 1;
                for (int q = 0; q < cnt[k]; ++q) prod *= sc[idx[off[k] + q]];
                V += prod;
            }
            const Wd a = first ? V : acc[p] + V;
            acc[p] = a;
            tv = (Wd)mu[p] * a;
        }
        tvs[t] = tv;
        __syncthreads();
        if (t == 0) {
            const int cntp = min(256, pe - p0);
            for (int q = 0; q < cntp; ++q) {
                U += tvs[q];
                const double td = (double)tvs[q];
                S += td < 0 ? -td : td;
            }
        }
        __syncthreads();
    }
    if (last && t == 0) {
        static_cast<Wd *>(uout)[ds] = U;
        sout[ds] = S;
    }
}

// Slice sources, 64 x 64 tiles through LDS so that both orientations read
// and write whole rows.
template <int DOM>
__global__ __launch_bounds__(256) void k_slicesrc(const SliceDesc *__restrict__ D, int nprob) {
    typedef typename Dom<DOM>::acc A;
    __shared__ A tile[64][65];
    const int64_t b = blockIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, b));  // uniform
    const SliceDesc &d = D[p];
    const int64_t local = b - d.tile_start;
    const int64_t ti = local / d.tiles, tu = local % d.tiles;
    const int64_t n = d.n, i0 = ti * 64, u0 = tu * 64;
    const int t = threadIdx.x;
    const MatRef m = d.src;
    for (int e = t; e < 4096; e += 256) {
        int r = e >> 6, c = e & 63;
        // trans == 0: element (i0 + r, u0 + c) at row i; trans == 1: element
        // (u0 + r, i0 + c) of the stored matrix, i.e. slice i0 + c, entry u0 + r
        int64_t a = (m.trans ? u0 : i0) + r, bb = (m.trans ? i0 : u0) + c;
        A x = (a < n && bb < n) ? load_elem<DOM>(m.p, m.dtype, a * m.ld + bb) : (A)0;
        if (m.trans) tile[c][r] = x;
        else tile[r][c] = x;
    }
    __syncthreads();
    for (int e = t; e < 4096; e += 256) {
        int r = e >> 6, c = e & 63;  // slice i0 + r, entry u0 + c
        int64_t i = i0 + r, u = u0 + c;
        if (i >= n || u >= n) continue;
        A x = tile[r][c];
        for (int q = 0; q < d.nscale; ++q) x *= load_vec<DOM>(d.scale[q], i);
        static_cast<A *>(d.out)[i * n + u] = x;
        if constexpr (DOM == DOM_INT) {
            if (d.mx_out) atomicMax(d.mx_out, (unsigned long long)(x < 0 ? -x : x));
        }
    }
}

// ----------------------------------------------------------------- launchers

hipError_t launch_rbf(const double *X, int64_t n, int32_t d, double divisor, void *out,
                      int32_t dtype, hipStream_t s) {
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 63) / 64));
    if (dtype == DT_F64)
        hipLaunchKernelGGL(k_rbf<double>, grid, dim3(256), 0, s, X, n, d, 1.0 / divisor,
                           static_cast<double *>(out));
    else
        hipLaunchKernelGGL(k_rbf<float>, grid, dim3(256), 0, s, X, n, d, 1.0 / divisor,
                           static_cast<float *>(out));
    return hipGetLastError();
}

hipError_t launch_diag(const DiagDesc *d, int nprob, int64_t max_n, int domain, hipStream_t s) {
    dim3 grid((unsigned)std::min<int64_t>(64, (max_n + 255) / 256), (unsigned)nprob);
    if (domain == DOM_FP) hipLaunchKernelGGL(k_diag<DOM_FP>, grid, dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL(k_diag<DOM_INT>, grid, dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

hipError_t launch_elim1(const Elim1Desc *d, int nprob, int64_t total_tiles, int domain,
                        hipStream_t s) {
    dim3 grid((unsigned)total_tiles);
    if (domain == DOM_FP) hipLaunchKernelGGL(k_elim1<DOM_FP>, grid, dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL(k_elim1<DOM_INT>, grid, dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

template <int DOM, typename T, int NM>
static void launch_colred_t(const ColDesc *d, int nprob, dim3 grid, int nout, bool rows,
                            hipStream_t s) {
    if (rows) {
        if (nout <= 4) hipLaunchKernelGGL((k_rowred<DOM, T, NM, 4>), grid, dim3(256), 0, s, d, nprob);
        else hipLaunchKernelGGL((k_rowred<DOM, T, NM, kColOut>), grid, dim3(256), 0, s, d, nprob);
        return;
    }
    if (nout <= 4) hipLaunchKernelGGL((k_colred<DOM, T, NM, 4>), grid, dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL((k_colred<DOM, T, NM, kColOut>), grid, dim3(256), 0, s, d, nprob);
}

template <int DOM, typename T>
static hipError_t launch_colred_nm(const ColDesc *d, int nprob, dim3 grid, int nm, int nout,
                                   bool rows, hipStream_t s) {
    switch (nm) {
        case 1: launch_colred_t<DOM, T, 1>(d, nprob, grid, nout, rows, s); break;
        case 2: launch_colred_t<DOM, T, 2>(d, nprob, grid, nout, rows, s); break;
        case 3: launch_colred_t<DOM, T, 3>(d, nprob, grid, nout, rows, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_colred(const ColDesc *d, int nprob, int64_t total_tiles, int nm, int max_out,
                         int elem_dtype, int domain, bool rows, hipStream_t s) {
    dim3 grid((unsigned)total_tiles);
    if (domain == DOM_INT)
        return launch_colred_nm<DOM_INT, void>(d, nprob, grid, nm, max_out, rows, s);
    if (elem_dtype == DT_F32)
        return launch_colred_nm<DOM_FP, float>(d, nprob, grid, nm, max_out, rows, s);
    if (elem_dtype == DT_F64)
        return launch_colred_nm<DOM_FP, double>(d, nprob, grid, nm, max_out, rows, s);
    return launch_colred_nm<DOM_FP, void>(d, nprob, grid, nm, max_out, rows, s);
}

hipError_t launch_reduce(const ReduceDesc *d, int nprob, int64_t max_len, int domain,
                         hipStream_t s) {
    dim3 grid((unsigned)nprob, (unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (max_len + 63) / 64)));
    if (domain == DOM_FP) hipLaunchKernelGGL(k_reduce<DOM_FP>, grid, dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL(k_reduce<DOM_INT>, grid, dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

hipError_t launch_elim0(const Elim0Desc *d, int nprob, int domain, hipStream_t s) {
    if (domain == DOM_FP) hipLaunchKernelGGL(k_elim0<DOM_FP>, dim3(nprob), dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL(k_elim0<DOM_INT>, dim3(nprob), dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

hipError_t launch_transpose(const TransDesc *d, int nprob, int64_t total_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)total_tiles), dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepDesc *d, int nprob, int64_t total_tiles, int domain,
                       hipStream_t s) {
    dim3 grid((unsigned)total_tiles);
    if (domain == DOM_FP) hipLaunchKernelGGL(k_prep<DOM_FP>, grid, dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL(k_prep<DOM_INT>, grid, dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

template <int PREC, class SH>
static hipError_t launch_gemm_t(const GemmDesc *d, int nprob, int64_t total_tiles, hipStream_t s) {
    size_t lds = (size_t)2 * gemm_stage_bytes<PREC, SH>();
    size_t red = (size_t)SH::NT * 16;
    if (lds < red) lds = red;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_gemm<PREC, SH>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_gemm<PREC, SH>), dim3((unsigned)total_tiles), dim3(SH::NT), lds, s, d,
                       nprob);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmDesc *d, int nprob, int64_t total_tiles, int precision,
                       int tile, hipStream_t s) {
    if (tile == 256) {
        if (precision == 1) return launch_gemm_t<1, S256>(d, nprob, total_tiles, s);
        if (precision == 2) return launch_gemm_t<2, S256>(d, nprob, total_tiles, s);
        return hipErrorInvalidValue;
    }
    switch (precision) {
        case 0: return launch_gemm_t<0, S128>(d, nprob, total_tiles, s);
        case 1: return launch_gemm_t<1, S128>(d, nprob, total_tiles, s);
        case 2: return launch_gemm_t<2, S128>(d, nprob, total_tiles, s);
        default: return launch_gemm_t<3, S128>(d, nprob, total_tiles, s);
    }
}

hipError_t launch_absmax_i8(const int8_t *const *src, const int64_t *n, int nprob,
                            unsigned long long *mx, hipStream_t s) {
    hipLaunchKernelGGL(k_absmax_i8, dim3(64, (unsigned)nprob), dim3(256), 0, s, src, n, nprob, mx);
    return hipGetLastError();
}

hipError_t launch_slicesrc(const SliceDesc *d, int nprob, int64_t total_tiles, int domain,
                           hipStream_t s) {
    if (domain == DOM_FP)
        hipLaunchKernelGGL(k_slicesrc<DOM_FP>, dim3((unsigned)total_tiles), dim3(256), 0, s, d, nprob);
    else
        hipLaunchKernelGGL(k_slicesrc<DOM_INT>, dim3((unsigned)total_tiles), dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineDesc *d, int ndata, const int32_t *term_off,
                          const int32_t *term_cnt, const int32_t *scal_off,
                          const int32_t *scal_cnt, const int32_t *scal_idx, const int64_t *mu,
                          const void *scal, void *acc, int first, int last, void *uout,
                          double *sout, int domain, hipStream_t s) {
    if (ndata <= 0) return hipSuccess;
    dim3 grid((unsigned)ndata);
    if (domain == DOM_FP)
        hipLaunchKernelGGL(k_combine<DOM_FP>, grid, dim3(256), 0, s, d, ndata, term_off, term_cnt,
                           scal_off, scal_cnt, scal_idx, mu, scal, acc, first, last, uout, sout);
    else
        hipLaunchKernelGGL(k_combine<DOM_INT>, grid, dim3(256), 0, s, d, ndata, term_off, term_cnt,
                           scal_off, scal_cnt, scal_idx, mu, scal, acc, first, last, uout, sout);
    return hipGetLastError();
}

}  // namespace ustat
