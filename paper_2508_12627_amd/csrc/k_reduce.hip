// Column and row reductions (degree-1 eliminations), fixed-order partial
// reductions and degree-0 eliminations.
//
// Every reduction is performed in a fixed order (per-tile partials written
// to memory, then summed in increasing tile index), so results are bitwise
// reproducible; no floating-point atomics are used anywhere.

#include "kdev.hpp"

namespace ustat {


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
        unsigned long long mxl = 0;  // largest |out[j]| written by this thread
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
                    const unsigned long long a = (unsigned long long)(s < 0 ? -s : s);
                    mxl = a > mxl ? a : mxl;
                }
            }
            __syncthreads();
        }
        if constexpr (DOM == DOM_INT) {
            if (d.mx_out) block_atomic_max(d.mx_out, mxl);
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

hipError_t launch_elim1(const Elim1Desc *d, int nprob, int64_t total_tiles, int domain,
                        hipStream_t s) {
    dim3 grid((unsigned)total_tiles);
    if (domain == DOM_FP) hipLaunchKernelGGL(k_elim1<DOM_FP>, grid, dim3(256), 0, s, d, nprob);
    else hipLaunchKernelGGL(k_elim1<DOM_INT>, grid, dim3(256), 0, s, d, nprob);
    return hipGetLastError();
}

hipError_t launch_colred(const ColDesc *d, int nprob, int64_t total_tiles, int nm, int max_out,
                         int elem_dtype, int domain, bool rows, hipStream_t s) {
    dim3 grid((unsigned)total_tiles);
    if (domain == DOM_INT)
        return rows ? launch_rowred_dt<DOM_INT, void>(d, nprob, grid, nm, max_out, s)
                    : launch_colred_dt<DOM_INT, void>(d, nprob, grid, nm, max_out, s);
    if (elem_dtype == DT_F32)
        return rows ? launch_rowred_dt<DOM_FP, float>(d, nprob, grid, nm, max_out, s)
                    : launch_colred_dt<DOM_FP, float>(d, nprob, grid, nm, max_out, s);
    if (elem_dtype == DT_F64)
        return rows ? launch_rowred_dt<DOM_FP, double>(d, nprob, grid, nm, max_out, s)
                    : launch_colred_dt<DOM_FP, double>(d, nprob, grid, nm, max_out, s);
    return rows ? launch_rowred_dt<DOM_FP, void>(d, nprob, grid, nm, max_out, s)
                : launch_colred_dt<DOM_FP, void>(d, nprob, grid, nm, max_out, s);
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

}  // namespace ustat
