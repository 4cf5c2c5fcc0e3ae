// Column-mode grouped reductions (degree-1 eliminations): kernel template
// and its launcher; the instantiations live in k_colred_*.hip.

#pragma once

#include "kdev.hpp"

namespace ustat {


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


template <int DOM, typename T>
hipError_t launch_colred_dt(const ColDesc *d, int nprob, dim3 grid, int nm, int nout, hipStream_t s) {
    switch (nm) {
        case 1:
            if (nout <= 4) hipLaunchKernelGGL((k_colred<DOM, T, 1, 4>), grid, dim3(256), 0, s, d, nprob);
            else hipLaunchKernelGGL((k_colred<DOM, T, 1, kColOut>), grid, dim3(256), 0, s, d, nprob);
            break;
        case 2:
            if (nout <= 4) hipLaunchKernelGGL((k_colred<DOM, T, 2, 4>), grid, dim3(256), 0, s, d, nprob);
            else hipLaunchKernelGGL((k_colred<DOM, T, 2, kColOut>), grid, dim3(256), 0, s, d, nprob);
            break;
        case 3:
            if (nout <= 4) hipLaunchKernelGGL((k_colred<DOM, T, 3, 4>), grid, dim3(256), 0, s, d, nprob);
            else hipLaunchKernelGGL((k_colred<DOM, T, 3, kColOut>), grid, dim3(256), 0, s, d, nprob);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


}  // namespace ustat
