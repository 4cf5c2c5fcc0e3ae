// GEMM steps on MFMA (gfx950): operand tiles staged through LDS, fp64,
// fp32, split-bf16 and int8-limb products, stored or fused with their
// consumer.

#include "kdev.hpp"

namespace ustat {

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
    static constexpr int BK = 128, PLANES = 1;
};
template <>
struct GemmCfg<kGemmBf16x6> {  // bf16 hi/mid/lo
    typedef uint16_t E;
    static constexpr int BK = 32, PLANES = 3;
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
//
// Split-bf16 (two planes) interleaves the planes instead: a 128-byte LDS row
// holds the row's hi chunks 0..3 and lo chunks 4..7, XOR-swizzled as
// chunk ^ (row & 7).  Measured on gfx950 (rocprofv3 SQ_LDS_BANK_CONFLICT),
// 16-byte fragment reads of 16 rows x 4 chunks conflict whatever the
// permutation inside 64-byte rows, and not at all over 128-byte rows
// swizzled this way.  int8 limbs use the same 128-byte rows with one plane
// (128 values of k per row, two MFMA k-steps of 64).
template <int PREC, int R, int NT>
struct TileIO {
    typedef GemmCfg<PREC> C;
    static constexpr int ROWB = C::BK * (int)sizeof(typename C::E);  // bytes per row
    static constexpr int UPR = ROWB / 16;                            // 16B units per row
    static constexpr int UNITS = R * UPR * C::PLANES;
    static constexpr int PER = UNITS / NT;
    static_assert(UNITS % NT == 0, "tile units must divide over the threads");
    static constexpr bool ILV = PREC == 2 || PREC == 3;  // 128-byte rows, planes interleaved
    static constexpr int LROW = (PREC == 0) ? ROWB + 16 : ILV ? C::PLANES * ROWB : ROWB;
    static_assert(!ILV || LROW == 128, "interleaved rows are 128 bytes");
    static constexpr int PLANEB = ILV ? 4 * 16 : R * LROW;  // plane offset: in chunks*16 when ILV
    static constexpr int STAGE = ILV ? R * LROW : PLANEB * C::PLANES;

    __device__ static __forceinline__ int off(int row, int chunk) {
        if constexpr (PREC == 0) return row * LROW + chunk * 16;
        else if constexpr (ILV) return row * LROW + ((chunk ^ (row & 7)) << 4);
        else return row * LROW + ((chunk ^ ((row >> 1) & 3) ^ ((row >> 3) & 1)) << 4);
    }
    // The 16-byte unit a thread moves: plane-major in general; row-major
    // with the planes of a row adjacent when they are interleaved, so that
    // consecutive lanes fill whole 128-byte LDS rows.
    __device__ static __forceinline__ void unit(int u, int &pl, int &row, int &cu) {
        if constexpr (ILV) {
            row = u / (C::PLANES * UPR);
            pl = (u / UPR) % C::PLANES;
            cu = u % UPR;
        } else {
            pl = u / (R * UPR);
            const int uu = u % (R * UPR);
            row = uu / UPR;
            cu = uu % UPR;
        }
    }
    // LDS offset of 16-byte chunk `chunk` of plane `pl` in row `row`
    __device__ static __forceinline__ int poff(int pl, int row, int chunk) {
        if constexpr (ILV) return off(row, pl * UPR + chunk);
        else return pl * PLANEB + off(row, chunk);
    }
    __device__ static void load(u32x4 (&r)[PER], const char *base, int64_t ldb, int64_t planeb,
                                int64_t row0, int64_t k0b) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int pl, row, cu;
            unit(threadIdx.x + NT * i, pl, row, cu);
            const char *g = base + (uint32_t)(pl * planeb + (row0 + row) * ldb + k0b + cu * 16);
            // a 32-bit offset from the uniform base (every operand buffer is
            // below 4 GiB, checked when the schedule is built); global address space:
            // these loads only count against vmcnt, so waiting for LDS
            // fragment reads never waits for the prefetch
            r[i] = *(const __attribute__((address_space(1))) u32x4 *)(g);
        }
    }
    // Direct-to-LDS staging of the interleaved layout (global_load_lds,
    // 16 bytes per lane): a wave instruction fills 8 consecutive 128-byte
    // LDS rows, lane l landing at slot l (row l / 8, position l % 8); the
    // lane loads the plane and chunk that the swizzle puts at that position.
    // Wave wv issues instructions wv, wv + NW, ... of the tile.
    static constexpr int DMA_PER = R / 8 / (NT / 64);
    __device__ static void dma(const char *base, int64_t ldb, int64_t planeb, int64_t row0,
                               int64_t k0b, char *lds) {
        static_assert(ILV && R % (8 * (NT / 64)) == 0, "direct staging: interleaved rows");
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int pos = lane & 7;
#pragma unroll
        for (int q = 0; q < DMA_PER; ++q) {
            const int r0 = (wv + (NT / 64) * q) * 8;
            const int row = r0 + (lane >> 3);
            const int c8 = pos ^ (row & 7);
            const int pl = c8 / UPR, cu = c8 % UPR;
            const char *g = base + (uint32_t)(pl * planeb + (row0 + row) * ldb + k0b + cu * 16);
            __builtin_amdgcn_global_load_lds((const void *)g,
                                             (__attribute__((address_space(3))) void *)(lds + r0 * LROW),
                                             16, 0, 0);
        }
    }
    __device__ static void store(const u32x4 (&r)[PER], char *lds) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int pl, row, cu;
            unit(threadIdx.x + NT * i, pl, row, cu);
            *reinterpret_cast<u32x4 *>(lds + poff(pl, row, cu)) = r[i];
        }
    }
};

// One BK step of a wave's FM x FN blocks: A rows from ra0, B rows from rb0
// (tile-local), fragments read from LDS with the staging layout of R-row
// tiles (the layout does not depend on R).
template <int PREC, int FM, int FN, int RA, int RB, bool OVERLAP = true>
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
        // Row-block major: the B fragments and row block 0's A fragments
        // first, then per row block its 3 FN products while the next row
        // block's A fragments are read (the scheduling groups below keep
        // that interleave, so LDS latency hides behind MFMAs).  For each
        // (i, j) the small cross terms come first, then hi*hi; the products
        // of one accumulator are FN instructions apart.
        bf16x8 bh[FN], bl[FN], ah[FM], al[FM];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            bh[j] = *reinterpret_cast<const bf16x8 *>(Bs + IOB::poff(0, rb0 + j * 16 + lr, lg));
            bl[j] = *reinterpret_cast<const bf16x8 *>(Bs + IOB::poff(1, rb0 + j * 16 + lr, lg));
        }
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            ah[i] = *reinterpret_cast<const bf16x8 *>(As + IOA::poff(0, ra0 + i * 16 + lr, lg));
            al[i] = *reinterpret_cast<const bf16x8 *>(As + IOA::poff(1, ra0 + i * 16 + lr, lg));
        }
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
        // scheduling groups: DS reads of B and row block 0, then for each
        // row block its MFMAs with the next row block's two reads
        __builtin_amdgcn_sched_group_barrier(0x100, 2 * FN + 2, 0);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            if (i + 1 < FM) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 3 * FN, 0);
        }
    } else if constexpr (PREC == kGemmBf16x6) {
        // the six products of order 1, 2^-9 and 2^-18 of a three-plane
        // split (a0 + a1 + a2)(b0 + b1 + b2), smallest first; the three
        // dropped ones are of order 2^-27 and below
        bf16x8 b0[FN], b1[FN], b2[FN];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int rb = IOB::off(rb0 + j * 16 + lr, lg);
            b0[j] = *reinterpret_cast<const bf16x8 *>(Bs + rb);
            b1[j] = *reinterpret_cast<const bf16x8 *>(Bs + IOB::PLANEB + rb);
            b2[j] = *reinterpret_cast<const bf16x8 *>(Bs + 2 * IOB::PLANEB + rb);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const int ra = IOA::off(ra0 + i * 16 + lr, lg);
            const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(As + ra);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(As + IOA::PLANEB + ra);
            const bf16x8 a2 = *reinterpret_cast<const bf16x8 *>(As + 2 * IOA::PLANEB + ra);
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0[j], acc[i][j], 0, 0, 0);
            }
        }
    } else {
        // two k-steps of 64: 16-byte chunks 0..3 of the row, then 4..7.  With
        // OVERLAP the second step's fragments are read while the first one's
        // MFMAs run (16 more live registers: used where the wide sums of
        // several limb passes are not live, which would spill)
        i32x4 a[2][FM], b[2][FN];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[ks][j] = *reinterpret_cast<const i32x4 *>(Bs + IOB::off(rb0 + j * 16 + lr, 4 * ks + lg));
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[ks][i] = *reinterpret_cast<const i32x4 *>(As + IOA::off(ra0 + i * 16 + lr, 4 * ks + lg));
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[ks][i], b[ks][j], acc[i][j], 0, 0, 0);
        // scheduling groups: the first step's reads, then its MFMAs two at a
        // time with one read of the second step between, then the rest
        if constexpr (OVERLAP) {
            __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
#pragma unroll
            for (int q = 0; q < FM + FN; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, FM * FN / (FM + FN), 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
        } else {
            // each step's reads just before its MFMAs
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
            }
        }
    }
}

// LDS bytes of one double-buffered (A, B) stage pair for a shape.
template <int PREC, class SH>
constexpr int gemm_stage_bytes() {
    return TileIO<PREC, SH::BM, SH::NT>::STAGE + TileIO<PREC, SH::BN, SH::NT>::STAGE;
}

// K loop of the interleaved layouts over K steps [k0, k1): the next K tile
// goes from global memory straight into the idle LDS buffer (no register
// staging, no LDS stores), issued at the top of the step; its completion and
// one barrier end the step.  Buffer parity counts from k0.
template <int PREC, class SH, bool OVERLAP = true>
__device__ __forceinline__ void gemm_range_dma(typename AccT<PREC>::T (&acc)[SH::FM][SH::FN],
                                               const char *Ab, const char *Bb, int64_t ldb,
                                               int64_t planeb, int64_t w0, int64_t x0, int64_t k0,
                                               int64_t k1, char *lds) {
    typedef TileIO<PREC, SH::BM, SH::NT> IOA;
    typedef TileIO<PREC, SH::BN, SH::NT> IOB;
    constexpr int PAIR = IOA::STAGE + IOB::STAGE;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ra0 = (wv / SH::WN) * SH::FM * 16, rb0 = (wv % SH::WN) * SH::FN * 16;
    constexpr int KB = GemmCfg<PREC>::BK * (int)sizeof(typename GemmCfg<PREC>::E);
    IOA::dma(Ab, ldb, planeb, w0, k0 * KB, lds);
    IOB::dma(Bb, ldb, planeb, x0, k0 * KB, lds + IOA::STAGE);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int64_t kt = k0; kt < k1; ++kt) {
        const int cur = (int)((kt - k0) & 1);
        char *As = lds + cur * PAIR;
        char *Bs = As + IOA::STAGE;
        char *An = lds + (1 - cur) * PAIR;
        // the last step re-reads its own tile into the idle buffer, which
        // keeps the loop free of branches
        const int64_t kn = (kt + 1 < k1) ? kt + 1 : kt;
        IOA::dma(Ab, ldb, planeb, w0, kn * KB, An);
        IOB::dma(Bb, ldb, planeb, x0, kn * KB, An + IOA::STAGE);
        __builtin_amdgcn_sched_barrier(0);
        mma_tile<PREC, SH::FM, SH::FN, SH::BM, SH::BN, OVERLAP>(acc, As, Bs, ra0, rb0, lane);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

template <int PREC, class SH, bool OVERLAP = true>
__device__ __forceinline__ void gemm_pass_dma(typename AccT<PREC>::T (&acc)[SH::FM][SH::FN],
                                              const char *Ab, const char *Bb, int64_t ldb,
                                              int64_t planeb, int64_t w0, int64_t x0, int64_t npad,
                                              char *lds) {
    gemm_range_dma<PREC, SH, OVERLAP>(acc, Ab, Bb, ldb, planeb, w0, x0, 0,
                                      npad / GemmCfg<PREC>::BK, lds);
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
        if constexpr (PREC == 1 || PREC == 2 || PREC == kGemmBf16x6) __builtin_amdgcn_sched_barrier(0);
        mma_tile<PREC, SH::FM, SH::FN, SH::BM, SH::BN>(acc, As, Bs, ra0, rb0, lane);
        if constexpr (PREC == 1 || PREC == 2 || PREC == kGemmBf16x6) __builtin_amdgcn_sched_barrier(0);
        char *An = lds + (1 - cur) * PAIR;
        IOA::store(ra, An);
        IOB::store(rb, An + IOA::STAGE);
        __syncthreads();
    }
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
        // Limb pair (la, lb) carries weight 2^(7 (la + lb)).  The first pass
        // (weight 1) initialises the wide sums, so they are not live during
        // its K loop; only products of multi-limb operands run the others.
        const int nla = d.la_p ? *d.la_p : d.la, nlb = d.lb_p ? *d.lb_p : d.lb;
        const char *Ab = static_cast<const char *>(d.A), *Bb = static_cast<const char *>(d.B);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = AT{0, 0, 0, 0};
        gemm_pass_dma<PREC, SH>(acc, Ab, Bb, ldb, planeb, w0, x0, d.npad, lds);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) resi[i][j][r] = (long long)acc[i][j][r];
        for (int q = 1; q < nla * nlb; ++q) {
            const int la = q / nlb, lb = q - (q / nlb) * nlb;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = AT{0, 0, 0, 0};
            gemm_pass_dma<PREC, SH, false>(acc, Ab + la * planeb, Bb + lb * planeb, ldb, planeb,
                                           w0, x0, d.npad, lds);
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
        if constexpr (TileIO<PREC, SH::BM, SH::NT>::ILV)
            gemm_pass_dma<PREC, SH>(acc, static_cast<const char *>(d.A), static_cast<const char *>(d.B),
                                    ldb, planeb, w0, x0, d.npad, lds);
        else
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
                block_atomic_max(d.mx_out, mloc);
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

// ---------------------------------------------------------- symmetric products

// Store a finished tile (I, J), I <= J, of C = P P^T (fp32) and, off the
// diagonal, its mirror (J, I): lane l holds column x = ... + l % 16 and the
// four consecutive rows 4 (l / 16) + r, which the mirror writes as one
// 16-byte store into row x.
template <int PREC, class SH>
__device__ __forceinline__ void sym_store(const typename AccT<PREC>::T (&acc)[SH::FM][SH::FN],
                                          const GemmDesc &d, int64_t I, int64_t J) {
    static_assert(PREC == 2, "symmetric products: split-bf16 with fp32 output");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wr0 = I * SH::BM + (wv / SH::WN) * SH::FM * 16;
    const int64_t xc0 = J * SH::BN + (wv % SH::WN) * SH::FN * 16;
    float *const C = static_cast<float *>(d.C);
    const int64_t ldc = d.ldc, n = d.n;
    const bool vec = (n % 4) == 0 && (ldc % 4) == 0;
#pragma unroll
    for (int i = 0; i < SH::FM; ++i)
#pragma unroll
        for (int j = 0; j < SH::FN; ++j) {
            const int64_t x = xc0 + j * 16 + (lane & 15);
            const int64_t wb = wr0 + i * 16 + 4 * (lane >> 4);
            if (x >= n) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (wb + r < n) C[(wb + r) * ldc + x] = acc[i][j][r];
            if (I == J) continue;
            if (vec) {
                if (wb < n) *reinterpret_cast<f32x4 *>(C + x * ldc + wb) = acc[i][j];
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (wb + r < n) C[x * ldc + wb + r] = acc[i][j][r];
            }
        }
}

// Owner (block) of unit u when `units` are cut into G ranges
// [floor(b units / G), floor((b + 1) units / G)).
__device__ __forceinline__ int64_t sym_owner(int64_t u, int64_t units, int64_t G) {
    return ((u + 1) * G - 1) / units;
}

template <int PREC, class SH>
__global__ __launch_bounds__(SH::NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_gemm_sym(const GemmDesc *__restrict__ D, int nprob, int64_t units, float *__restrict__ part) {
    typedef typename AccT<PREC>::T AT;
    constexpr int FM = SH::FM, FN = SH::FN, NT = SH::NT;
    constexpr int ES = (int)sizeof(typename GemmCfg<PREC>::E);
    extern __shared__ __align__(16) char lds[];
    const int64_t G = gridDim.x;
    const int64_t lb = xcd_remap(blockIdx.x, G);  // neighbouring ranges share an XCD
    const int64_t u0 = lb * units / G, u1 = (lb + 1) * units / G;
    if (u0 >= u1) return;
    // first unit of the tile holding unit u
    auto tile_first = [&](int64_t u) {
        const GemmDesc &d = D[find_problem(D, nprob, u)];
        const int64_t nk = d.npad / GemmCfg<PREC>::BK;
        return d.tile_start + (u - d.tile_start) / nk * nk;
    };
    // The range's last piece (the start of a tile, K from 0) goes first and
    // the rest follow: all blocks then stand at one of two K positions at any
    // time, which keeps the operand slices being read few (cache reuse).
    const int64_t ul = tile_first(u1 - 1) > u0 ? tile_first(u1 - 1) : u0;
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t ua = pass == 0 ? ul : u0, ub = pass == 0 ? u1 : ul;
        for (int64_t u = ua; u < ub;) {
            const int p = __builtin_amdgcn_readfirstlane(find_problem(D, nprob, u));  // uniform
            const GemmDesc &d = D[p];
            const int64_t nk = d.npad / GemmCfg<PREC>::BK;
            const int64_t lu = u - d.tile_start;
            const int64_t t = lu / nk, k0 = lu - t * nk;
            const int64_t k1 = (k0 + (ub - u) < nk) ? k0 + (ub - u) : nk;
            int64_t I, J;
            sym_tile(t, d.tiles, I, J);
            AT acc[FM][FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = AT{0, 0, 0, 0};
            const int64_t ldb = d.ld * ES, planeb = d.plane * ES;
            gemm_range_dma<PREC, SH>(acc, static_cast<const char *>(d.A),
                                     static_cast<const char *>(d.B), ldb, planeb, I * SH::BM,
                                     J * SH::BN, k0, k1, lds);
            if (k0 == 0 && k1 == nk) {
                sym_store<PREC, SH>(acc, d, I, J);
            } else {
                AT *P = reinterpret_cast<AT *>(part);
                const int64_t slot = 2 * lb + (u == u0 ? 0 : 1);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        P[slot * (FM * FN * NT) + (i * FN + j) * NT + threadIdx.x] = acc[i][j];
            }
            u += k1 - k0;
        }
    }
}

// Fix-up of a symmetric-product launch, one block per tile of the launch:
// a tile whose units fell to more than one block is the sum of their pieces,
// added in block order (slot 2 b when the piece holds block b's first unit,
// else 2 b + 1), then stored with its mirror.
template <int PREC, class SH>
__global__ __launch_bounds__(SH::NT) void k_gemm_symfix(const GemmDesc *__restrict__ D, int nprob,
                                                        int64_t units, int64_t G,
                                                        const float *__restrict__ part) {
    typedef typename AccT<PREC>::T AT;
    constexpr int FM = SH::FM, FN = SH::FN, NT = SH::NT;
    const int64_t gt = blockIdx.x;
    int lo = 0, hi = nprob - 1;  // the problem owning tile gt
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (D[mid].sym_tile0 <= gt) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc &d = D[lo];
    const int64_t t = gt - d.sym_tile0, nk = d.npad / GemmCfg<PREC>::BK;
    const int64_t tf = d.tile_start + t * nk;
    const int64_t bf = sym_owner(tf, units, G), bl = sym_owner(tf + nk - 1, units, G);
    if (bf == bl) return;  // stored whole by the product kernel
    const AT *P = reinterpret_cast<const AT *>(part);
    AT acc[FM][FN];
    for (int64_t b = bf; b <= bl; ++b) {
        const int64_t sb = 2 * b + (b * units / G >= tf ? 0 : 1);
        const AT *Q = P + sb * (FM * FN * NT);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const AT v = Q[(i * FN + j) * NT + threadIdx.x];
                acc[i][j] = b == bf ? v : acc[i][j] + v;
            }
    }
    int64_t I, J;
    sym_tile(t, d.tiles, I, J);
    sym_store<PREC, SH>(acc, d, I, J);
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
        case 3: return launch_gemm_t<3, S128>(d, nprob, total_tiles, s);
        case kGemmBf16x6: return launch_gemm_t<kGemmBf16x6, S128>(d, nprob, total_tiles, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_sym(const GemmDesc *d, int nprob, int64_t units, int blocks, int64_t tiles,
                           float *part, hipStream_t s) {
    static_assert(S256::FM * S256::FN * 4 * S256::NT == kSymSlot, "partial slot size");
    const size_t lds = (size_t)2 * gemm_stage_bytes<2, S256>();
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_gemm_sym<2, S256>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_gemm_sym<2, S256>), dim3((unsigned)blocks), dim3(S256::NT), lds, s, d,
                       nprob, units, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gemm_symfix<2, S256>), dim3((unsigned)tiles), dim3(S256::NT), 0, s, d,
                       nprob, units, (int64_t)blocks, (const float *)part);
    return hipGetLastError();
}

}  // namespace ustat
