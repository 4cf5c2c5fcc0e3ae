// Row-mode grouped reductions (degree-1 eliminations over symmetric
// matrices): kernel template and its launcher; the instantiations live in
// k_rowred_*.hip, one translation unit per element type.

#pragma once

#include "kdev.hpp"

namespace ustat {



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
    // [output][q][j][lane]: with four outputs exactly 32 KB, which lets a
    // block share a compute unit with a 128 KB GEMM block
    __shared__ A svt[NOUT * SEGMAX];
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
    // each wave's row sums: lane r holds those of its row r
    A mine[NOUT];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) mine[o] = 0;
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
                if (lane == r) mine[o] = acc;
            }
        }
    };
    if (vecld) run(std::true_type{});
    else run(std::false_type{});
    const int64_t w = wrow0 + lane;
    if (lane < RPW && w < n) {
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
            if (o < nout) ((__attribute__((address_space(1))) A *)(d.o[o].part))[ts * n + w] = mine[o];
    }
}

template <int DOM, typename T>
hipError_t launch_rowred_dt(const ColDesc *d, int nprob, dim3 grid, int nm, int nout, hipStream_t s) {
    switch (nm) {
        case 1:
            if (nout <= 4) hipLaunchKernelGGL((k_rowred<DOM, T, 1, 4>), grid, dim3(256), 0, s, d, nprob);
            else hipLaunchKernelGGL((k_rowred<DOM, T, 1, kColOut>), grid, dim3(256), 0, s, d, nprob);
            break;
        case 2:
            if (nout <= 4) hipLaunchKernelGGL((k_rowred<DOM, T, 2, 4>), grid, dim3(256), 0, s, d, nprob);
            else hipLaunchKernelGGL((k_rowred<DOM, T, 2, kColOut>), grid, dim3(256), 0, s, d, nprob);
            break;
        case 3:
            if (nout <= 4) hipLaunchKernelGGL((k_rowred<DOM, T, 3, 4>), grid, dim3(256), 0, s, d, nprob);
            else hipLaunchKernelGGL((k_rowred<DOM, T, 3, kColOut>), grid, dim3(256), 0, s, d, nprob);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


}  // namespace ustat
