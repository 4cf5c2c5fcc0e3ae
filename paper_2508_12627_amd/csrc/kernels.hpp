// Device kernels of the elimination engine and their grouped-launch
// descriptors.  Every kernel takes an array of descriptors, one per
// independent problem, so that all steps of one dependency level of every
// restricted V-statistic (and every dataset of a batch) go out in a single
// launch per step kind.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ustat {

enum DType : int32_t { DT_F64 = 0, DT_F32 = 1, DT_I8 = 2, DT_I64 = 3 };

// Accumulation domain of a launch: floating point (double) or exact
// integers (int64 values, 128-bit scalars).
enum Domain : int32_t { DOM_FP = 0, DOM_INT = 1 };

constexpr int kMaxMat = 12;  // matrices per Hadamard group
constexpr int kMaxVec = 12;  // vectors multiplied on one variable

// Matrix operand addressed in its step's canonical orientation (a, b):
// trans == 0 reads p[a*ld + b], trans == 1 reads p[b*ld + a].  zdiag
// zeroes entries with a == b (sparsified input factors, Lemma 3).
struct MatRef {
    const void *p;
    int64_t ld;
    int32_t dtype;
    int32_t trans;
    int32_t zdiag;
    int32_t pad;
};

// dst[i] = src(i, i), as double (DOM_FP) or int64 (DOM_INT).
struct DiagDesc {
    MatRef src;
    void *dst;
    int64_t n;
    unsigned long long *mx_out;  // DOM_INT: running max |dst|, or null
};

// Strip partials of y(w) = sum_v prod_k A_k(v, w) prod_j s_j(v) with every
// operand stored (v, w) (trans == 0): part[tv * n + w] holds the sum over
// rows [tv*strip, (tv+1)*strip) for the 256 columns of strip tw;
// tiles_v = ceil(n / strip), tiles_w = ceil(n / 256).
struct Elim1Desc {
    int64_t n;
    int32_t nA, nS;
    MatRef A[kMaxMat];
    const void *s[kMaxVec];
    void *part;
    int64_t tile_start;  // first block index of this problem in the launch
    int32_t tiles_v, tiles_w;
    int32_t strip;       // rows per block (a multiple of 32)
};

// Grouped column reductions over the same few matrices: for every output o
// of the group, y_o(w) = sum_v prod_k M_k(v,w)^e[o][k] prod_j s_oj(v), with
// the k-th factor taken as 0 on the diagonal where zd[o][k].  Each element
// of each distinct matrix is read once for all outputs.  Partials as for
// Elim1Desc, one buffer per output; strips and tiles as there.
constexpr int kColMat = 3;  // distinct matrices per group
constexpr int kColOut = 8;  // outputs per group
struct ColOut {
    int8_t e[kColMat];
    int8_t zd[kColMat];
    int32_t nS;
    const void *s[kMaxVec];
    void *part;
};
struct ColDesc {
    int64_t n;
    int32_t nm, nout;
    MatRef M[kColMat];  // stored (v, w)
    ColOut o[kColOut];
    int64_t tile_start;
    int32_t tiles_v, tiles_w;
    int32_t strip;  // rows per block (a multiple of 32)
    // 1: every matrix is symmetric and the reduction runs along rows w:
    // blocks of kRowBlock rows by `strip` columns (256, 512 or 1024),
    // tiles_v column segments (one partial each) times tiles_w row blocks
    int32_t rows;
};

// out[j] = (sum_{t < T} part[t * stride + j]) * prod_q mul_q[j], j < len,
// summed in increasing t (fixed order).  With `dot` set, the len products
// are summed as well (fixed order) into the single scalar out[0].
struct ReduceDesc {
    const void *part;
    int64_t T, len, stride;
    void *out;
    int32_t nmul, dot;
    const void *mul[kMaxVec];
    unsigned long long *mx_out;  // DOM_INT vectors: running max |out|, or null
};

// Materialised transpose: dst[b * n + a] = src[a * ld + b], a, b < n, in
// 64 x 64 tiles (tiles = ceil(n / 64) per side).
struct TransDesc {
    const void *src;
    void *dst;
    int64_t n, ld;
    int32_t dtype, tiles;
    int64_t tile_start;
};

// out = sum_v prod_j s_j(v) (one block per problem).
struct Elim0Desc {
    int64_t n;
    int32_t nS;
    const void *s[kMaxVec];
    void *out;
};

enum PrepFormat : int32_t { PF_F64 = 0, PF_F32 = 1, PF_BF16X2 = 2, PF_I8LIMBS = 3, PF_BF16X3 = 4 };

// Padded size of the GEMM operands of an n x n matrix in prep format fmt:
// fp32 and two-plane split-bf16 operands from n = 1024 on are padded to a
// multiple of 256 so that their products can take 256-wide tiles; all
// others to a multiple of 128.
inline int64_t gemm_npad(int64_t n, int fmt) {
    const int64_t a = (n >= 1024 && (fmt == PF_F32 || fmt == PF_BF16X2)) ? 256 : 128;
    return (n + a - 1) / a * a;
}

// GEMM operand: out[w * ldo + v] = prod_j s_j(v) prod_k A_k(v, w) for
// w, v < n and 0 in the padding up to npad, every operand stored (w, v)
// (trans == 1); tiles of 64 rows x 128 columns, (npad/64) * (npad/128) per
// problem; ldo a multiple of 4.  PF_BF16X2 writes hi at out and
// lo at out + plane (elements); PF_BF16X3 writes hi, mid and lo planes
// (x - hi - mid rounded); PF_I8LIMBS writes `limbs` planes of 7-bit
// digits (balanced for all but the top one).
struct PrepDesc {
    int64_t n, npad, ldo, plane;
    int32_t nA, nS;
    MatRef A[kMaxMat];
    const void *s[kMaxVec];
    void *out;
    int32_t format, limbs;  // limbs: planes available (PF_I8LIMBS)
    int64_t tile_start;
    int32_t tiles;  // per side, over npad
    int32_t nmx;
    // PF_I8LIMBS: the digit count is chosen on the device from the product
    // of the operands' running maxima mx[0..nmx) and written to *limbs_out.
    const unsigned long long *mx[kMaxMat + kMaxVec];
    int32_t *limbs_out;
};

// C(w, x) = sum_v Aop[w][v] * Bop[x][v] over prepared operands (leading
// dimension ld, zero-padded to npad).  final == 0 stores C (n x n, ldc) as
// dtype_c; final == 1 writes per-tile partials of
//   sum_{w,x} C(w,x) prod_k Z_k(w,x) prod aw(w) prod bx(x).
struct GemmDesc {
    int64_t n, npad, ld;
    const void *A;
    const void *B;
    int64_t plane;       // elements between limb / lo planes
    int32_t la, lb;      // limb counts (int8 path)
    int32_t final_, dtype_c;
    void *C;
    int64_t ldc;
    int32_t nZ, naw, nbx, tiles;  // tiles per side
    MatRef Z[kMaxMat];
    const void *aw[kMaxVec];
    const void *bx[kMaxVec];
    void *part;
    int64_t tile_start;
    const int32_t *la_p, *lb_p;  // int8 path: limb counts written by prep
    unsigned long long *mx_out;  // int8 path: running max |C|, or null
    int64_t sym_tile0;           // symmetric products: first tile of the problem in the launch
};

// Per dataset d, for its programs p in order:
//   V_p = sum over terms t of p (in order) of prod_j scal[term scalars],
//   acc[p] = (first ? 0 : acc[p]) + V_p,
// and when `last`: U_d = sum_p mu_p acc[p], S_d = sum_p |mu_p acc[p]|.
// A program conditioned on one vertex has one term per slice; slices may
// arrive over several launches (chunks), accumulated in acc in chunk order.
// DOM_FP scalars are doubles; DOM_INT scalars are int128.
struct CombineDesc {
    int32_t p_begin, p_end;  // V-statistics of this dataset
};

// Slice source for conditioning: out[i * n + u] = M(i, u) (trans == 0) or
// M(u, i) (trans == 1), times prod_q scale_q[i]; accumulation type output.
struct SliceDesc {
    MatRef src;
    int32_t nscale, tiles;
    const void *scale[kMaxVec];
    void *out;
    int64_t n, tile_start;
    unsigned long long *mx_out;  // DOM_INT: running max |out|, or null
};

constexpr int kGemmTile = 128;
constexpr int kTile = 64;
constexpr int kElimStrip = 512;  // largest rows per column-reduction block
constexpr int kRowBlock = 32;  // rows per row-mode reduction block (four waves)
// Columns per row-mode block for size n: 256 columns per 64 lanes of
// float4 loads, up to four groups.
inline int row_segment(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return g >= 4 ? 1024 : g >= 2 ? 512 : 256;
}

// Rows per column-reduction block for size n: about 1024 blocks per
// problem (so that even a single problem fills the chip), in multiples of
// 32 rows, between 32 and kElimStrip.
inline int elim_strip_rows(int64_t n) {
    const int64_t wstrips = (n + 255) / 256;
    int64_t s = (n * wstrips / 1024) / 32 * 32;
    if (s < 32) s = 32;
    if (s > kElimStrip) s = kElimStrip;
    return (int)s;
}

// RBF factor (n x n, dtype DT_F64 or DT_F32) and, when op is non-null, its
// GEMM-operand form in prep format op_format (PF_F64 with DT_F64; PF_F32 or
// PF_BF16X2 with DT_F32), npad = ceil(n / 128) * 128, zero padded.
hipError_t launch_rbf(const double *X, int64_t n, int32_t d, double divisor, void *out,
                      int32_t dtype, hipStream_t s, void *op = nullptr, int32_t op_format = -1);
hipError_t launch_diag(const DiagDesc *d, int nprob, int64_t max_n, int domain, hipStream_t s);
hipError_t launch_elim1(const Elim1Desc *d, int nprob, int64_t total_tiles, int domain,
                        hipStream_t s);
// nm: the number of distinct matrices of every group in d (1..kColMat);
// max_out: the largest output count of a group; elem_dtype: the DType of
// every matrix of the launch, or -1 when they differ; rows: every group is
// in row mode (ColDesc::rows), else none is
hipError_t launch_colred(const ColDesc *d, int nprob, int64_t total_tiles, int nm, int max_out,
                         int elem_dtype, int domain, bool rows, hipStream_t s);
hipError_t launch_reduce(const ReduceDesc *d, int nprob, int64_t max_len, int domain,
                         hipStream_t s);
hipError_t launch_elim0(const Elim0Desc *d, int nprob, int domain, hipStream_t s);
hipError_t launch_transpose(const TransDesc *d, int nprob, int64_t total_tiles, hipStream_t s);
hipError_t launch_prep(const PrepDesc *d, int nprob, int64_t total_tiles, int domain,
                       hipStream_t s);
// precision: a ustat_precision, or kGemmBf16x6 for split-bf16 operands
// prepared in three planes (PF_BF16X3) whose products take the six terms
// of order up to 2^-18 (128-wide tiles only).
// tile: 128 (any precision) or 256 (fp32 and two-plane split-bf16;
// npad % 256 == 0, GemmDesc::tiles counted in 256-row tiles)
constexpr int kGemmBf16x6 = 4;
hipError_t launch_gemm(const GemmDesc *d, int nprob, int64_t total_tiles, int precision,
                       int tile, hipStream_t s);

// Symmetric products C = P P^T (the same prepared split-bf16 operand on both
// sides, fp32 output, 256-wide tiles): only the tiles (I, J) with I <= J are
// computed, in the order of sym_tile, and each one off the diagonal is also
// stored mirrored at (J, I).  A problem is t (t + 1) / 2 tiles (t =
// GemmDesc::tiles) of nk = npad / 32 K steps each, "units";
// GemmDesc::tile_start is its first unit in the launch and sym_tile0 its
// first tile.  The launch's `units` are cut into `blocks` equal ranges, one
// per block (stream-K).  A block stores a tile it covers entirely; a piece
// of a tile goes to partial slot 2 b (the piece holding the block's first
// unit) or 2 b + 1 (its last), kSymSlot floats each, and a second kernel
// (one block per tile of the launch, `tiles` in all) adds each split
// tile's pieces in block order and stores it.
constexpr int kSymBlocks = 256;                 // compute units of the MI355X
constexpr int64_t kSymSlot = 256 * 256;         // floats per partial slot
// Tile t of the order in which symmetric products visit the tiles (I, J),
// I <= J, of a t_side x t_side grid: 4 x 4 groups of tiles, row by row over
// the groups on and above the diagonal, column by column inside a group, so
// that the blocks running at the same time (consecutive ranges of the order)
// share few operand panels.  Used by the kernel and by the host layout.
__host__ __device__ inline void sym_tile(int64_t t, int64_t t_side, int64_t &I, int64_t &J) {
    const int64_t g = (t_side + 3) / 4;
    I = J = 0;
    for (int64_t P = 0; P < g; ++P)
        for (int64_t Q = P; Q < g; ++Q) {
            const int64_t r0 = 4 * P, r1 = (4 * P + 4 < t_side) ? 4 * P + 4 : t_side;
            const int64_t c0 = 4 * Q, c1 = (4 * Q + 4 < t_side) ? 4 * Q + 4 : t_side;
            for (int64_t c = c0; c < c1; ++c) {
                const int64_t hi = (r1 < c + 1) ? r1 : c + 1;  // rows I <= c of the group
                const int64_t k = hi > r0 ? hi - r0 : 0;
                if (t < k) {
                    I = r0 + t;
                    J = c;
                    return;
                }
                t -= k;
            }
        }
}
hipError_t launch_gemm_sym(const GemmDesc *d, int nprob, int64_t units, int blocks, int64_t tiles,
                           float *part, hipStream_t s);

// Peak microbenchmarks (k_peak.hip).  launch_peak_mfma: `blocks` blocks of
// four waves, each issuing `iters` rounds of eight independent MFMAs of one
// kind (0 bf16 16x16x32, 1 fp64 16x16x4, 2 int8 16x16x64, 3 fp32 16x16x4);
// *flops receives the operations launched; sink: kPeakSinkSlots x 32 bytes
// of device memory.  launch_peak_copy: a streaming copy of `bytes` (a
// multiple of 16) from src to dst.
constexpr int kPeakSinkSlots = 4096;
hipError_t launch_peak_mfma(int kind, int blocks, int64_t iters, char *sink, hipStream_t s,
                            double *flops);
hipError_t launch_peak_copy(const void *src, void *dst, int64_t bytes, int blocks, hipStream_t s);
// flag[p] = 1 when matrix p (n[p] x n[p], fp32 when f32 else fp64) holds a
// negative (or NaN) entry, else 0; the flags must be zero on entry.
hipError_t launch_signscan(const void *const *src, const int64_t *n, int nprob, int f32,
                           unsigned int *flag, hipStream_t s);
// B = 1 - A off the diagonal and 0 on it (n x n int8); *hbad (host)
// receives nonzero when A is not a symmetric 0/1 matrix with a zero
// diagonal; dbad is device scratch.  Synchronises s.
hipError_t launch_motif_complement(const int8_t *A, int8_t *B, int64_t n, unsigned int *dbad,
                                   unsigned int *hbad, hipStream_t s);
// mx[p] = max |entry| of int8 matrix p, mx[nprob + p] = 1 if it has a
// negative entry (mx zeroed by the caller, 2 nprob words).
hipError_t launch_absmax_i8(const int8_t *const *src, const int64_t *n, int nprob,
                            unsigned long long *mx, hipStream_t s);
hipError_t launch_slicesrc(const SliceDesc *d, int nprob, int64_t total_tiles, int domain,
                           hipStream_t s);
hipError_t launch_combine(const CombineDesc *d, int ndata, const int32_t *term_off,
                          const int32_t *term_cnt, const int32_t *scal_off,
                          const int32_t *scal_cnt, const int32_t *scal_idx, const int64_t *mu,
                          const void *scal, void *acc, int first, int last, void *uout,
                          double *sout, int domain, hipStream_t s);

}  // namespace ustat
