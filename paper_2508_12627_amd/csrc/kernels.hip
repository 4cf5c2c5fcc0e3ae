// HIP kernels for gfx950 (CDNA4): factor build, diagonals, transposes,
// operand preparation, slice sources and the Moebius combination.
//
// Every reduction is performed in a fixed order (per-tile partials written
// to memory, then summed in increasing tile index), so results are bitwise
// reproducible; no floating-point atomics are used anywhere.

#include "kdev.hpp"

namespace ustat {

// ----------------------------------------------------------------- RBF

// RBF factor K(i,j) = exp(-||x_i - x_j||^2 / divisor) (Algorithm 1 with the
// kernel on an edge as the factor).  The squared distance comes from the
// Gram matrix on fp64 MFMA (16x16x4): ||x_i||^2 + ||x_j||^2 - 2 x_i.x_j,
// clamped at 0, with the norms summed over the coordinates in increasing
// order; K(i,i) = 1 exactly.  Only 64 x 64 tiles on or above the diagonal
// are computed; each value is written at (i, j) and, staged through LDS, at
// (j, i), so K is symmetric bit for bit.  With OPF >= 0 the same values are
// also written in the GEMM-operand form of that prep format (npad x npad,
// zero padded: fp64, fp32, or bf16 hi and lo planes), so that no separate
// operand preparation of the factor is needed.
// Stores one 64 x 64 tile of the factor (rows r0.., columns c0..) from the
// LDS tile, transposed when `mirror`.  Every store instruction of a wave
// writes whole 16-byte pieces of consecutive rows (16 lanes per fp32 row of
// 64 values, 8 lanes per row of a bf16 plane), so each row segment is
// written by adjacent lanes of one instruction; the LDS reads of both
// orientations stay free of bank conflicts (row pitch 65 words).
template <typename KT, int OPF>
__device__ __forceinline__ void rbf_store_tile(KT *__restrict__ K, void *__restrict__ op, int64_t n,
                                               int64_t npad, int64_t r0, int64_t c0,
                                               const KT (&val)[64][65], bool mirror) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int t = threadIdx.x;
    auto at = [&](int r, int c) -> KT { return mirror ? val[c][r] : val[r][c]; };
    {
        constexpr int PER = 16 / (int)sizeof(KT), LPR = 64 / PER;
        const bool vec = n % PER == 0;
#pragma unroll
        for (int it = 0; it < 64 * LPR / 256; ++it) {
            const int idx = it * 256 + t, r = idx / LPR, c = (idx % LPR) * PER;
            const int64_t g = r0 + r, col = c0 + c;
            if (g >= n) continue;
            KT *dst = K + g * n + col;
            if (vec && col + PER <= n) {
                if constexpr (sizeof(KT) == 4)
                    *reinterpret_cast<f32x4 *>(dst) = f32x4{at(r, c), at(r, c + 1), at(r, c + 2), at(r, c + 3)};
                else
                    *reinterpret_cast<d2 *>(dst) = d2{at(r, c), at(r, c + 1)};
            } else {
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    if (col + e < n) dst[e] = at(r, c + e);
            }
        }
    }
    // the operand form covers npad x npad: every row and column of the tile
    if constexpr (OPF == PF_F64) {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int idx = it * 256 + t, r = idx >> 5, c = (idx & 31) * 2;
            double *o = static_cast<double *>(op) + (r0 + r) * npad + c0 + c;
            *reinterpret_cast<d2 *>(o) = d2{(double)at(r, c), (double)at(r, c + 1)};
        }
    } else if constexpr (OPF == PF_F32) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int idx = it * 256 + t, r = idx >> 4, c = (idx & 15) * 4;
            float *o = static_cast<float *>(op) + (r0 + r) * npad + c0 + c;
            *reinterpret_cast<f32x4 *>(o) = f32x4{(float)at(r, c), (float)at(r, c + 1),
                                                  (float)at(r, c + 2), (float)at(r, c + 3)};
        }
    } else if constexpr (OPF == PF_BF16X2) {
        // the split of the fp32 factor value, as the operand preparation
        // forms it: hi = bf16(x), lo = bf16(x - hi)
        typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = it * 256 + t, r = idx >> 3, c = (idx & 7) * 8;
            u16x8 hi, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const double xd = (double)(float)at(r, c + e);
                const uint16_t h = f32_to_bf16_rne((float)xd);
                hi[e] = h;
                lo[e] = f32_to_bf16_rne((float)(xd - (double)bf16_to_f32(h)));
            }
            uint16_t *o = static_cast<uint16_t *>(op) + (r0 + r) * npad + c0 + c;
            *reinterpret_cast<u16x8 *>(o) = hi;
            *reinterpret_cast<u16x8 *>(o + npad * npad) = lo;
        }
    }
}

template <typename KT, int OPF>
__global__ __launch_bounds__(256) void k_rbf(const double *__restrict__ X, int64_t n, int32_t d,
                                             double inv_div, KT *__restrict__ K,
                                             void *__restrict__ op, int64_t npad) {
    if (blockIdx.y > blockIdx.x) return;  // lower-triangle tiles come from the mirror
    // coordinates of the tile's i and j samples, 16 at a time; values staged
    // in the factor's element type (what is written anyway): about 35 KB for
    // fp32 factors, so that four blocks share a compute unit
    __shared__ double xs[2][64][17];
    __shared__ double nrm[2][64];
    __shared__ KT val[64][65];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int qi = wv >> 1, qj = wv & 1;  // the wave's 32 x 32 quadrant
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    double nacc = 0.0;  // threads < 128: squared norm of one sample
    for (int k0 = 0; k0 < d; k0 += 16) {
        // clamped loads, all in flight together; entries outside the samples
        // or coordinates are zeroed afterwards
        double v[8];
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = t + 256 * it, side = e >> 10, rr = (e >> 4) & 63, kk = e & 15;
            const int64_t g = (side ? j0 : i0) + rr;
            v[it] = X[min(g, n - 1) * d + min(k0 + kk, d - 1)];
        }
        if (k0 > 0) __syncthreads();  // the previous chunk's reads are done
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = t + 256 * it, side = e >> 10, rr = (e >> 4) & 63, kk = e & 15;
            const int64_t g = (side ? j0 : i0) + rr;
            xs[side][rr][kk] = (g < n && k0 + kk < d) ? v[it] : 0.0;
        }
        __syncthreads();
        if (t < 128) {
            const int side = t >> 6, rr = t & 63;
            for (int kk = 0; kk < 16; ++kk) nacc = fma(xs[side][rr][kk], xs[side][rr][kk], nacc);
        }
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = xs[0][qi * 32 + a * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = xs[1][qj * 32 + b * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    if (t < 128) nrm[t >> 6][t & 63] = nacc;
    __syncthreads();
    // item r of lane l in a 16 x 16 block of the fp64 MFMA: row l/16 + 4 r,
    // column l % 16
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = qi * 32 + a * 16 + (lane >> 4) + 4 * r;
                const int col = qj * 32 + b * 16 + (lane & 15);
                const int64_t gi = i0 + row, gj = j0 + col;
                double sq = nrm[0][row] + nrm[1][col] - 2.0 * acc[a][b][r];
                sq = sq > 0.0 ? sq : 0.0;
                const double k = gi == gj ? 1.0 : exp(-sq * inv_div);
                val[row][col] = (KT)((gi < n && gj < n) ? k : 0.0);
            }
    __syncthreads();
    rbf_store_tile<KT, OPF>(K, op, n, npad, i0, j0, val, false);
    if (blockIdx.x == blockIdx.y) return;  // the diagonal tile is its own mirror
    rbf_store_tile<KT, OPF>(K, op, n, npad, j0, i0, val, true);
}

// ----------------------------------------------------------------- diag

template <int DOM>
__global__ void k_diag(const DiagDesc *__restrict__ D, int nprob) {
    const DiagDesc &d = D[blockIdx.y];
    unsigned long long mxl = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        typedef typename Dom<DOM>::acc A;
        A v = load_elem<DOM>(d.src.p, d.src.dtype, i * d.src.ld + i);
        static_cast<A *>(d.dst)[i] = v;
        if constexpr (DOM == DOM_INT) {
            const unsigned long long a = (unsigned long long)(v < 0 ? -v : v);
            mxl = a > mxl ? a : mxl;
        }
    }
    if constexpr (DOM == DOM_INT) {
        if (d.mx_out) block_atomic_max(d.mx_out, mxl);
    }
}

// Sign scan of fp32 or fp64 matrices: flag[p] is set when matrix p holds a
// negative entry (or a NaN, for which no sign can be relied on).  Loads are
// issued from clamped indices, four per thread per round.
template <typename T>
__global__ __launch_bounds__(256) void k_signscan(const void *const *src, const int64_t *n,
                                                  int nprob, unsigned int *flag) {
    const int p = blockIdx.y;
    const T *a = static_cast<const T *>(src[p]);
    const int64_t cnt = n[p] * n[p];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool neg = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += 4 * stride) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = a[min(i + u * stride, cnt - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) neg = neg || !(v[u] >= (T)0);
    }
    if (__any(neg) && (threadIdx.x & 63) == 0) atomicOr(&flag[p], 1u);
}

// Complement of a simple graph's adjacency for motif kernels: B = 1 - A off
// the diagonal, 0 on it, in 64 x 64 tiles; the tile and its mirror go
// through LDS so that *bad is set (once per wave) when A is not a symmetric
// 0/1 matrix with a zero diagonal.
__global__ __launch_bounds__(256) void k_motif_complement(const int8_t *__restrict__ A,
                                                          int8_t *__restrict__ B, int64_t n,
                                                          unsigned int *bad) {
    __shared__ int8_t ta[64][65], tb[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int t = threadIdx.x;
    for (int e = t; e < 4096; e += 256) {
        const int r = e >> 6, c = e & 63;
        const int64_t i = i0 + r, j = j0 + c;
        ta[r][c] = (i < n && j < n) ? A[i * n + j] : (int8_t)0;
        const int64_t i2 = j0 + r, j2 = i0 + c;  // the mirror tile, row-major
        tb[r][c] = (i2 < n && j2 < n) ? A[i2 * n + j2] : (int8_t)0;
    }
    __syncthreads();
    bool wrong = false;
    for (int e = t; e < 4096; e += 256) {
        const int r = e >> 6, c = e & 63;
        const int64_t i = i0 + r, j = j0 + c;
        if (i >= n || j >= n) continue;
        const int a = ta[r][c], at = tb[c][r];
        wrong = wrong || (a != 0 && a != 1) || a != at || (i == j && a != 0);
        B[i * n + j] = (int8_t)(i == j ? 0 : 1 - a);
    }
    if (__any(wrong) && (t & 63) == 0) atomicOr(bad, 1u);
}

hipError_t launch_motif_complement(const int8_t *A, int8_t *B, int64_t n, unsigned int *dbad,
                                   unsigned int *hbad, hipStream_t s) {
    hipError_t e = hipMemsetAsync(dbad, 0, sizeof(unsigned int), s);
    if (e != hipSuccess) return e;
    const unsigned T = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_motif_complement, dim3(T, T), dim3(256), 0, s, A, B, n, dbad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(hbad, dbad, sizeof(unsigned int), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    return hipStreamSynchronize(s);
}

// Largest |entry| of int8 matrices (one running max per problem).
__global__ __launch_bounds__(256) void k_absmax_i8(const int8_t *const *src, const int64_t *n,
                                                    int nprob, unsigned long long *mx) {
    const int p = blockIdx.y;
    const int8_t *a = src[p];
    const int64_t cnt = n[p] * n[p];
    int best = 0, neg = 0;
    // 16 entries per load where the matrix allows it (hipMalloc'd buffers
    // are 256-byte aligned; cnt a multiple of 16), single bytes otherwise
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (((uintptr_t)a & 15) == 0 && (cnt & 15) == 0) {
        const uint4 *a16 = reinterpret_cast<const uint4 *>(a);
        for (int64_t i = t0; i < cnt / 16; i += stride) {
            const uint4 q = a16[i];
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int v = (int8_t)(w[k] >> (8 * b));
                    best = max(best, v < 0 ? -v : v);
                    neg |= v < 0;
                }
        }
    } else {
        for (int64_t i = t0; i < cnt; i += stride) {
            const int v = a[i];
            best = max(best, v < 0 ? -v : v);
            neg |= v < 0;
        }
    }
    __shared__ int red[256], rneg[256];
    red[threadIdx.x] = best;
    rneg[threadIdx.x] = neg;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0, ng = 0;
        for (int q = 0; q < 256; ++q) {
            m = max(m, red[q]);
            ng |= rneg[q];
        }
        atomicMax(&mx[p], (unsigned long long)m);
        if (ng) atomicMax(&mx[nprob + p], 1ull);
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
            case PF_BF16X3: {
                // x = hi + mid + lo + r with |r| below about 2^-26 |x|: each
                // plane rounds what the previous ones leave (in fp64, exact)
                typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
                u16x4 hi, mid, lo;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    double xd = (double)pr[i][j];
                    const uint16_t h = f32_to_bf16_rne((float)xd);
                    xd -= (double)bf16_to_f32(h);
                    const uint16_t md = f32_to_bf16_rne((float)xd);
                    xd -= (double)bf16_to_f32(md);
                    hi[j] = h;
                    mid[j] = md;
                    lo[j] = f32_to_bf16_rne((float)xd);
                }
                *reinterpret_cast<u16x4 *>(static_cast<uint16_t *>(out) + o) = hi;
                *reinterpret_cast<u16x4 *>(static_cast<uint16_t *>(out) + o + plane) = mid;
                *reinterpret_cast<u16x4 *>(static_cast<uint16_t *>(out) + o + 2 * plane) = lo;
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
    unsigned long long mxl = 0;
    for (int e = t; e < 4096; e += 256) {
        int r = e >> 6, c = e & 63;  // slice i0 + r, entry u0 + c
        int64_t i = i0 + r, u = u0 + c;
        if (i >= n || u >= n) continue;
        A x = tile[r][c];
        for (int q = 0; q < d.nscale; ++q) x *= load_vec<DOM>(d.scale[q], i);
        static_cast<A *>(d.out)[i * n + u] = x;
        if constexpr (DOM == DOM_INT) {
            const unsigned long long a = (unsigned long long)(x < 0 ? -x : x);
            mxl = a > mxl ? a : mxl;
        }
    }
    if constexpr (DOM == DOM_INT) {
        if (d.mx_out) block_atomic_max(d.mx_out, mxl);
    }
}

// ----------------------------------------------------------------- launchers

hipError_t launch_rbf(const double *X, int64_t n, int32_t d, double divisor, void *out,
                      int32_t dtype, hipStream_t s, void *op, int32_t op_format) {
    const int64_t npad = gemm_npad(n, op_format);
    const unsigned T = (unsigned)(op ? npad / 64 : (n + 63) / 64);
    dim3 grid(T, T);
    const double inv = 1.0 / divisor;
    if (dtype == DT_F64) {
        if (op && op_format == PF_F64)
            hipLaunchKernelGGL((k_rbf<double, PF_F64>), grid, dim3(256), 0, s, X, n, d, inv,
                               static_cast<double *>(out), op, npad);
        else if (!op)
            hipLaunchKernelGGL((k_rbf<double, -1>), grid, dim3(256), 0, s, X, n, d, inv,
                               static_cast<double *>(out), op, npad);
        else
            return hipErrorInvalidValue;
    } else {
        if (op && op_format == PF_F32)
            hipLaunchKernelGGL((k_rbf<float, PF_F32>), grid, dim3(256), 0, s, X, n, d, inv,
                               static_cast<float *>(out), op, npad);
        else if (op && op_format == PF_BF16X2)
            hipLaunchKernelGGL((k_rbf<float, PF_BF16X2>), grid, dim3(256), 0, s, X, n, d, inv,
                               static_cast<float *>(out), op, npad);
        else if (!op)
            hipLaunchKernelGGL((k_rbf<float, -1>), grid, dim3(256), 0, s, X, n, d, inv,
                               static_cast<float *>(out), op, npad);
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_diag(const DiagDesc *d, int nprob, int64_t max_n, int domain, hipStream_t s) {
    dim3 grid((unsigned)std::min<int64_t>(64, (max_n + 255) / 256), (unsigned)nprob);
    if (domain == DOM_FP) hipLaunchKernelGGL(k_diag<DOM_FP>, grid, dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL(k_diag<DOM_INT>, grid, dim3(256), 0, s, d, nprob);
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

hipError_t launch_signscan(const void *const *src, const int64_t *n, int nprob, int f32,
                           unsigned int *flag, hipStream_t s) {
    if (f32)
        hipLaunchKernelGGL(k_signscan<float>, dim3(256, (unsigned)nprob), dim3(256), 0, s, src, n, nprob, flag);
    else
        hipLaunchKernelGGL(k_signscan<double>, dim3(256, (unsigned)nprob), dim3(256), 0, s, src, n, nprob, flag);
    return hipGetLastError();
}

hipError_t launch_absmax_i8(const int8_t *const *src, const int64_t *n, int nprob,
                            unsigned long long *mx, hipStream_t s) {
    hipLaunchKernelGGL(k_absmax_i8, dim3(512, (unsigned)nprob), dim3(256), 0, s, src, n, nprob, mx);
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
