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
        double acc = 0.0;
        for (int64_t x = 0; x < st.nx; ++x) acc += lr_term(p, off, sx, nin, x);
        ws[st.out + o] = acc;
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
        for (int64_t x = x0 + xl; x < x1; x += st.xlanes) acc += lr_term(p, off, sx, nin, x);
    }
    red[tid] = acc;
    __syncthreads();
    if (xl == 0 && o < st.nout) {
        double s = red[ol];
        for (int j = 1; j < st.xlanes; ++j) s += red[ol + j * st.otile];
        ws[st.out + c * st.nout + o] = s;
    }
}

__global__ __launch_bounds__(kLrThreads) void k_lr_reduce(const LrReduceDesc *__restrict__ desc,
                                                          int64_t nred, double *__restrict__ ws) {
    const int64_t b = blockIdx.x;
    const LrReduceDesc &rd = desc[find_step(desc, nred, b)];
    const int64_t o = (b - rd.block0) * kLrThreads + threadIdx.x;
    if (o >= rd.nout) return;
    const double *p = ws + rd.part + o;
    double s = 0.0;
    for (int c = 0; c < rd.nchunk; ++c) s += p[c * rd.nout];
    ws[rd.out + o] = s;
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
