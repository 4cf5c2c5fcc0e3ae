// Kernels of the low-rank evaluation: one launch per dependency level runs
// every summation step of that level (each block finds its step by binary
// search over the steps' first blocks), a second sums the chunk partials of
// the steps over a sample index, and one block forms the Moebius
// combination of Lemma 2.  fp64 throughout.
#include <hip/hip_runtime.h>

#include "lowrank.hpp"

namespace ustat {

namespace {

template <typename D>
__device__ inline int64_t find_step(const D *__restrict__ d, int64_t nsteps, int64_t b) {
    int64_t lo = 0, hi = nsteps - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (d[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Input offsets of output o: base + sum_d digit_d(o) so[d].
__device__ inline void lr_offsets(const LrStepDesc &st, int64_t o, int64_t off[kLrMaxIn]) {
#pragma unroll
    for (int t = 0; t < kLrMaxIn; ++t) off[t] = st.base[t];
    if (st.nout <= 0xffffffffLL) {
        uint32_t rem = (uint32_t)o;
        for (int d = st.nd - 1; d >= 0; --d) {
            const uint32_t dm = (uint32_t)st.dim[d];
            const uint32_t q = rem / dm;
            const int64_t dig = rem - q * dm;
            rem = q;
#pragma unroll
            for (int t = 0; t < kLrMaxIn; ++t)
                if (t < st.nin) off[t] += dig * st.so[t][d];
        }
    } else {
        int64_t rem = o;
        for (int d = st.nd - 1; d >= 0; --d) {
            const int64_t q = rem / st.dim[d];
            const int64_t dig = rem - q * st.dim[d];
            rem = q;
#pragma unroll
            for (int t = 0; t < kLrMaxIn; ++t)
                if (t < st.nin) off[t] += dig * st.so[t][d];
        }
    }
}

__device__ inline double lr_term(const double *const p[kLrMaxIn], const int64_t off[kLrMaxIn],
                                 const int64_t sx[kLrMaxIn], int nin, int64_t x) {
    double prod = p[0][off[0] + x * sx[0]];
#pragma unroll
    for (int t = 1; t < kLrMaxIn; ++t)
        if (t < nin) prod *= p[t][off[t] + x * sx[t]];
    return prod;
}

__global__ __launch_bounds__(kLrThreads) void k_lr_steps(const LrStepDesc *__restrict__ desc,
                                                         int64_t nsteps,
                                                         const double *const *__restrict__ tab) {
    __shared__ double red[kLrThreads];
    const int64_t b = blockIdx.x;
    const LrStepDesc &st = desc[find_step(desc, nsteps, b)];
    const int64_t bi = b - st.block0;
    const int tid = threadIdx.x;
    const int nin = st.nin;
    const double *p[kLrMaxIn];
    int64_t sx[kLrMaxIn];
#pragma unroll
    for (int t = 0; t < kLrMaxIn; ++t) {
        p[t] = tab[t < nin ? st.slot[t] : 0];
        sx[t] = st.sx[t];
    }
    double *ws = const_cast<double *>(tab[0]);
    int64_t off[kLrMaxIn];
    if (st.mode == 0) {
        const int64_t o = bi * kLrThreads + tid;
        if (o >= st.nout) return;
        lr_offsets(st, o, off);
        // operand pointers formed once and stepped by their x strides; four
        // terms at a time in four sums (their loads in flight together),
        // added in a fixed order
        const double *q[kLrMaxIn];
#pragma unroll
        for (int t = 0; t < kLrMaxIn; ++t) q[t] = p[t] + off[t];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int64_t x = 0;
        for (; x + 3 < st.nx; x += 4) {
            double t0 = q[0][0], t1 = q[0][sx[0]], t2 = q[0][2 * sx[0]], t3 = q[0][3 * sx[0]];
#pragma unroll
            for (int t = 1; t < kLrMaxIn; ++t)
                if (t < nin) {
                    t0 *= q[t][0];
                    t1 *= q[t][sx[t]];
                    t2 *= q[t][2 * sx[t]];
                    t3 *= q[t][3 * sx[t]];
                }
            a0 += t0;
            a1 += t1;
            a2 += t2;
            a3 += t3;
#pragma unroll
            for (int t = 0; t < kLrMaxIn; ++t) q[t] += 4 * sx[t];
        }
        for (; x < st.nx; ++x) {
            double t0 = q[0][0];
#pragma unroll
            for (int t = 1; t < kLrMaxIn; ++t)
                if (t < nin) t0 *= q[t][0];
            a0 += t0;
#pragma unroll
            for (int t = 0; t < kLrMaxIn; ++t) q[t] += sx[t];
        }
        ws[st.out + o] = (a0 + a1) + (a2 + a3);
        return;
    }
    const int64_t tile = bi / st.nchunk, c = bi - tile * st.nchunk;
    const int ol = tid % st.otile, xl = tid / st.otile;
    const int64_t o = tile * st.otile + ol;
    const int64_t x0 = c * st.xchunk;
    const int64_t x1 = min(st.nx, x0 + st.xchunk);
    double acc = 0.0;
    if (o < st.nout) {
        lr_offsets(st, o, off);
        // two independent chains so that loads overlap
        double acc1 = 0.0;
        int64_t x = x0 + xl;
        for (; x + st.xlanes < x1; x += 2 * st.xlanes) {
            acc += lr_term(p, off, sx, nin, x);
            acc1 += lr_term(p, off, sx, nin, x + st.xlanes);
        }
        if (x < x1) acc += lr_term(p, off, sx, nin, x);
        acc += acc1;
    }
    red[tid] = acc;
    __syncthreads();
    if (xl == 0 && o < st.nout) {
        double s = red[ol];
        for (int j = 1; j < st.xlanes; ++j) s += red[ol + j * st.otile];
        ws[st.out + c * st.nout + o] = s;
    }
}

// Offset of index i of one side: sum_d digit_d(i) st[d], digits in radix
// dim[0..nd) with dim[nd-1] fastest (31-bit quantities).
__device__ inline uint32_t side_offset(uint32_t i, int nd, const int32_t *dim, const int32_t *st) {
    uint32_t off = 0;
    for (int d = nd - 1; d >= 0; --d) {
        const uint32_t dm = (uint32_t)dim[d];
        const uint32_t q = i / dm;
        off += (i - q * dm) * (uint32_t)st[d];
        i = q;
    }
    return off;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
// operands live in device global memory: global (not flat) loads
typedef const double __attribute__((address_space(1))) *gptr;

// Outer-product steps.  A 64 x 64 output tile per block of four waves (each
// wave a 32 x 32 sub-tile from 2 x 2 fp64 MFMA 16x16x4 blocks).  Per 16
// values of x the block forms the A and B operand tiles in LDS: thread t
// forms column t % 64 of both at rows t / 64 + 4q, each element the product
// of its side's operand reads at that x.  The raw reads of the next 16
// values are issued before the MFMAs of the current ones.  Tiles are
// k-major with a row pitch of 80 doubles, so the fragment reads of the two
// half-waves fall in different banks.  Rows and columns past M or N and x
// past the chunk read clamped (valid) addresses and are multiplied by zero.
constexpr int kKrBK = 16, kKrPitch = kLrKrTile + 16;

template <int NL, int NR>
__device__ __forceinline__ void kr_tile(const LrKrDesc &st, const double *const *__restrict__ tab,
                                        uint32_t c, uint32_t tm, uint32_t tn, double *As,
                                        double *Bs) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    const uint32_t il = tm * kLrKrTile + (tid & 63), ir = tn * kLrKrTile + (tid & 63);
    const double zl = il < (uint32_t)st.M ? 1.0 : 0.0, zr = ir < (uint32_t)st.N ? 1.0 : 0.0;
    const uint32_t ilc = min(il, (uint32_t)st.M - 1), irc = min(ir, (uint32_t)st.N - 1);
    gptr pl[NL], pr[NR];
    uint32_t ol[NL], orr[NR], sl[NL], sr[NR];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        pl[u] = (gptr)(tab[st.slot[u]] + st.base[u]);
        sl[u] = (uint32_t)st.sx[u];
        ol[u] = side_offset(ilc, st.ndl, st.dl, st.st[u]);
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        pr[u] = (gptr)(tab[st.slot[kLrKrSide + u]] + st.base[kLrKrSide + u]);
        sr[u] = (uint32_t)st.sx[kLrKrSide + u];
        orr[u] = side_offset(irc, st.ndr, st.dr, st.st[kLrKrSide + u]);
    }
    const uint32_t x0 = c * (uint32_t)st.xchunk;
    const uint32_t x1 = min((uint32_t)st.nx, x0 + (uint32_t)st.xchunk);
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
    double ra[kKrBK / 4][NL], rb[kKrBK / 4][NR];
    auto fetch = [&](uint32_t xb) {
#pragma unroll
        for (int q = 0; q < kKrBK / 4; ++q) {
            const uint32_t xc = min(xb + wv + 4 * q, x1 - 1);
#pragma unroll
            for (int u = 0; u < NL; ++u) ra[q][u] = pl[u][ol[u] + xc * sl[u]];
#pragma unroll
            for (int u = 0; u < NR; ++u) rb[q][u] = pr[u][orr[u] + xc * sr[u]];
        }
    };
    fetch(x0);
    for (uint32_t xb = x0; xb < x1; xb += kKrBK) {
#pragma unroll
        for (int q = 0; q < kKrBK / 4; ++q) {
            double a = xb + wv + 4 * q < x1 ? zl : 0.0, b = zr;
#pragma unroll
            for (int u = 0; u < NL; ++u) a *= ra[q][u];
#pragma unroll
            for (int u = 0; u < NR; ++u) b *= rb[q][u];
            As[(wv + 4 * q) * kKrPitch + (tid & 63)] = a;
            Bs[(wv + 4 * q) * kKrPitch + (tid & 63)] = b;
        }
        __syncthreads();
        fetch(xb + kKrBK);  // past x1: clamped reads, unused
        // keep those reads above the MFMAs (the scheduler would sink them
        // to their uses at the top of the next step)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = 0; kk < kKrBK; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[(kk + lg) * kKrPitch + wm + 16 * i + lr];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[(kk + lg) * kKrPitch + wn + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator element r of block (i, j): tile row wm + 16 i + lg + 4 r,
    // tile column wn + 16 j + lr
    double *o = const_cast<double *>(tab[0]) + st.out + (int64_t)c * st.nout;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const uint32_t col = tn * kLrKrTile + wn + 16 * j + lr;
        if (col >= (uint32_t)st.N) continue;
        const uint32_t co = side_offset(col, st.ndr, st.dr, st.orr);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t row = tm * kLrKrTile + wm + 16 * i + lg + 4 * r;
                if (row < (uint32_t)st.M) o[side_offset(row, st.ndl, st.dl, st.ol) + co] = acc[i][j][r];
            }
    }
}

// Outer-product steps with a short left side (at most 16 indices) and a
// right side of at most 64: no LDS staging.  For the fp64 MFMA 16x16x4 lane
// l holds A at (row l % 16, k l / 16) and B at (k l / 16, column l % 16), so
// each lane forms exactly those products: the left index l % 16 and the
// right indices 16 cb + l % 16 (cb < 4), at x = xq + l / 16.  The four
// waves take interleaved groups of four x values of the chunk, and their
// accumulators are added in wave order through LDS at the end.  Indices
// past the sides and x past the chunk read clamped addresses and are
// multiplied by zero.
template <int NS, int NW>
__device__ __forceinline__ void kr_small(const LrKrDesc &st, const double *const *__restrict__ tab,
                                         uint32_t c, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    constexpr int sb = 0, wb = kLrKrSide;  // short (left) and wide (right) operands
    const uint32_t MS = (uint32_t)st.M, MW = (uint32_t)st.N;
    const int nds = st.ndl, ndw = st.ndr;
    const int32_t *ds = st.dl, *dw = st.dr;
    const double zs = (uint32_t)lr < MS ? 1.0 : 0.0;
    const uint32_t isc = min((uint32_t)lr, MS - 1);
    gptr ps[NS], pw[NW];
    uint32_t os[NS], ss[NS], sw[NW], ow[4][NW];
    double zw[4];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        ps[u] = (gptr)(tab[st.slot[sb + u]] + st.base[sb + u]);
        ss[u] = (uint32_t)st.sx[sb + u];
        os[u] = side_offset(isc, nds, ds, st.st[sb + u]);
    }
#pragma unroll
    for (int u = 0; u < NW; ++u) {
        pw[u] = (gptr)(tab[st.slot[wb + u]] + st.base[wb + u]);
        sw[u] = (uint32_t)st.sx[wb + u];
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const uint32_t iw = 16 * cb + lr;
        zw[cb] = iw < MW ? 1.0 : 0.0;
#pragma unroll
        for (int u = 0; u < NW; ++u) ow[cb][u] = side_offset(min(iw, MW - 1), ndw, dw, st.st[wb + u]);
    }
    const int ncb = (int)((MW + 15) / 16);  // uniform
    const uint32_t x0 = c * (uint32_t)st.xchunk;
    const uint32_t x1 = min((uint32_t)st.nx, x0 + (uint32_t)st.xchunk);
    f64x4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = f64x4{0, 0, 0, 0};
    for (uint32_t xq = x0 + 4 * wv; xq < x1; xq += 16) {
        const uint32_t x = xq + lg;
        const uint32_t xc = min(x, x1 - 1);
        double a = x < x1 ? zs : 0.0;
#pragma unroll
        for (int u = 0; u < NS; ++u) a *= ps[u][os[u] + xc * ss[u]];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            if (cb >= ncb) break;
            double b = zw[cb];
#pragma unroll
            for (int u = 0; u < NW; ++u) b *= pw[u][ow[cb][u] + xc * sw[u]];
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
        }
    }
    // red[w][cb][r][lane]
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[((wv * 4 + cb) * 4 + r) * 64 + lane] = acc[cb][r];
    __syncthreads();
    double *o = const_cast<double *>(tab[0]) + st.out + (int64_t)c * st.nout;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int idx = tid + 256 * q;  // (cb, r, lane)
        const int cb = idx >> 8, r = (idx >> 6) & 3, l = idx & 63;
        // item r of lane l: left row l / 16 + 4 r, right column 16 cb + l % 16
        const uint32_t il = (uint32_t)((l >> 4) + 4 * r), ir = (uint32_t)(16 * cb + (l & 15));
        if (il >= MS || ir >= MW) continue;
        double v = red[((0 * 4 + cb) * 4 + r) * 64 + l];
#pragma unroll
        for (int w = 1; w < 4; ++w) v += red[((w * 4 + cb) * 4 + r) * 64 + l];
        o[side_offset(il, st.ndl, st.dl, st.ol) + side_offset(ir, st.ndr, st.dr, st.orr)] = v;
    }
}

__global__ __launch_bounds__(kLrThreads) void k_lr_kr(const LrKrDesc *__restrict__ desc,
                                                      int64_t nkr,
                                                      const double *const *__restrict__ tab) {
    // operand tiles of the 64 x 64 path, or the waves' sums of the small one
    __shared__ double lds[4 * 4 * 4 * 64];
    static_assert(2 * kKrBK * kKrPitch <= 4 * 4 * 4 * 64, "LDS of the 64 x 64 path");
    double *As = lds, *Bs = lds + kKrBK * kKrPitch;
    const int64_t b = blockIdx.x;
    const LrKrDesc &st = desc[find_step(desc, nkr, b)];
    const uint32_t bi = (uint32_t)(b - st.block0);
    const uint32_t c = bi / st.tiles, t = bi - c * st.tiles;
    const uint32_t tm = t / st.tiles_n, tn = t - tm * st.tiles_n;
    if (st.small) {
        switch (st.nl * 8 + st.nr) {
#define KS_CASE(S, W) \
    case S * 8 + W: kr_small<S, W>(st, tab, c, lds); break;
            KS_CASE(1, 1) KS_CASE(1, 2) KS_CASE(1, 3) KS_CASE(1, 4)
            KS_CASE(2, 1) KS_CASE(2, 2) KS_CASE(2, 3) KS_CASE(2, 4)
            KS_CASE(3, 1) KS_CASE(3, 2) KS_CASE(3, 3) KS_CASE(3, 4)
            KS_CASE(4, 1) KS_CASE(4, 2) KS_CASE(4, 3) KS_CASE(4, 4)
#undef KS_CASE
            default: break;
        }
        return;
    }
    switch (st.nl * 8 + st.nr) {
#define KR_CASE(L, R) \
    case L * 8 + R: kr_tile<L, R>(st, tab, c, tm, tn, As, Bs); break;
        KR_CASE(1, 1) KR_CASE(1, 2) KR_CASE(1, 3) KR_CASE(1, 4)
        KR_CASE(2, 1) KR_CASE(2, 2) KR_CASE(2, 3) KR_CASE(2, 4)
        KR_CASE(3, 1) KR_CASE(3, 2) KR_CASE(3, 3) KR_CASE(3, 4)
        KR_CASE(4, 1) KR_CASE(4, 2) KR_CASE(4, 3) KR_CASE(4, 4)
#undef KR_CASE
        default: break;
    }
}

__global__ __launch_bounds__(kLrThreads) void k_lr_reduce(const LrReduceDesc *__restrict__ desc,
                                                          int64_t nred, double *__restrict__ ws) {
    __shared__ double red[kLrThreads];
    const int64_t b = blockIdx.x;
    const LrReduceDesc &rd = desc[find_step(desc, nred, b)];
    const int tid = threadIdx.x;
    const int ol = tid % rd.otile, cl = tid / rd.otile;
    const int64_t o = (b - rd.block0) * rd.otile + ol;
    double s = 0.0;
    if (o < rd.nout) {
        const double *p = ws + rd.part + o;
        // two independent sums so that loads overlap
        double s1 = 0.0;
        int c = cl;
        for (; c + rd.clanes < rd.nchunk; c += 2 * rd.clanes) {
            s += p[(int64_t)c * rd.nout];
            s1 += p[(int64_t)(c + rd.clanes) * rd.nout];
        }
        if (c < rd.nchunk) s += p[(int64_t)c * rd.nout];
        s += s1;
    }
    red[tid] = s;
    __syncthreads();
    if (cl == 0 && o < rd.nout) {
        double t = red[ol];
        for (int j = 1; j < rd.clanes; ++j) t += red[ol + j * rd.otile];
        ws[rd.out + o] = t;
    }
}

__device__ inline void two_sum_add(double &s, double &c, double x) {
    // Neumaier's compensated addition
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

__global__ __launch_bounds__(kLrThreads) void k_lr_combine(const double *__restrict__ mu,
                                                           const double *__restrict__ cst,
                                                           const int32_t *__restrict__ first,
                                                           const int64_t *__restrict__ sc,
                                                           int nparts, const double *__restrict__ ws,
                                                           double *__restrict__ res) {
    __shared__ double sh[4][kLrThreads];
    const int tid = threadIdx.x;
    double s = 0, c = 0, a = 0, ac = 0;
    for (int p = tid; p < nparts; p += kLrThreads) {
        double v = cst[p];
        for (int k = first[p]; k < first[p + 1]; ++k) v *= ws[sc[k]];
        const double term = mu[p] * v;
        two_sum_add(s, c, term);
        two_sum_add(a, ac, fabs(term));
    }
    sh[0][tid] = s;
    sh[1][tid] = c;
    sh[2][tid] = a;
    sh[3][tid] = ac;
    __syncthreads();
    if (tid == 0) {
        double S = 0, C = 0, A = 0, AC = 0;
        for (int k = 0; k < kLrThreads; ++k) {
            two_sum_add(S, C, sh[0][k]);
            C += sh[1][k];
            two_sum_add(A, AC, sh[2][k]);
            AC += sh[3][k];
        }
        res[0] = S + C;
        res[1] = A + AC;
    }
}

}  // namespace

void launch_lr_steps(const LrStepDesc *d, int64_t nsteps, int64_t blocks,
                     const double *const *tab, hipStream_t s) {
    if (nsteps <= 0 || blocks <= 0) return;
    hipLaunchKernelGGL(k_lr_steps, dim3((unsigned)blocks), dim3(kLrThreads), 0, s, d, nsteps, tab);
}

void launch_lr_kr(const LrKrDesc *d, int64_t nkr, int64_t blocks, const double *const *tab,
                  hipStream_t s) {
    if (nkr <= 0 || blocks <= 0) return;
    hipLaunchKernelGGL(k_lr_kr, dim3((unsigned)blocks), dim3(kLrThreads), 0, s, d, nkr, tab);
}

void launch_lr_reduce(const LrReduceDesc *d, int64_t nred, int64_t blocks, double *ws,
                      hipStream_t s) {
    if (nred <= 0 || blocks <= 0) return;
    hipLaunchKernelGGL(k_lr_reduce, dim3((unsigned)blocks), dim3(kLrThreads), 0, s, d, nred, ws);
}

void launch_lr_combine(const double *mu, const double *cst, const int32_t *first,
                       const int64_t *sc, int nparts, const double *ws, double *res,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_lr_combine, dim3(1), dim3(kLrThreads), 0, s, mu, cst, first, sc, nparts,
                       ws, res);
}

}  // namespace ustat
