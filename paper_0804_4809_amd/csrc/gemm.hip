// Float64 MFMA GEMM for gfx950 and small memory-bound helpers.
//
// Every dense contraction of the method runs through this kernel: the Gram
// matrix A = G'G (Section 2, Eq. (1)), the panel updates of the full-rank
// Cholesky (Appendix loop), L'L, and the product chain L M M L' G'
// (Theorem 1).  Column-major operands, optional transposes, device-resident
// dimensions (the rank r), a lower-triangle-only mode for symmetric outputs
// and split-K for skinny products.
//
// Tiling: a workgroup owns a BM x BN tile of C, made of WM x WN wavefronts
// (64 lanes each); each wavefront owns (BM/WM) x (BN/WN) and issues
// v_mfma_f64_16x16x4_f64 on 16 x 16 blocks.  K is consumed in chunks of BK
// staged through double-buffered LDS; the next chunk's global loads are in
// flight while the current chunk feeds the matrix cores.  dgemm_kernel does
// this through registers (64 x 64 tiles, small and skinny products);
// dgemm_dma_kernel (128 x 128 tiles, the large products) loads straight into
// LDS.  Operands are read
// as 16-byte pairs from per-thread 32-bit offsets computed once, against a
// chunk origin that is the only thing that moves (few vector instructions per
// load: the address arithmetic was what held the matrix cores back).
//
// Two-level summation: the matrix-core accumulators only ever hold the sum
// over KFLUSH consecutive k; they are then added into a second set of
// float64 registers and restarted.  A single running sum over the whole
// K = m of the Gram matrix loses about sqrt(m/KFLUSH) times more accuracy,
// and the pseudoinverse amplifies Gram rounding by about cond(G)^4.
//
// MFMA operand roles are swapped (the instruction computes the transposed
// tile C' = op(B)' op(A)') so that the 16 lanes of a row group hold 16
// consecutive rows of one column of C: every store of the epilogue is a
// 128-byte contiguous run of the column-major output.
//
// Lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950): operand A
// element (i, k) in lane i + 16k, operand B element (k, j) in lane j + 16k,
// result element (i, j) in lane j + 16 (i % 4), accumulator slot i / 4.
#include "common.h"

#include <cstdint>
#include <cstdlib>

namespace geninv {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int KFLUSH = 256;

typedef double d2 __attribute__((ext_vector_type(2)));

// Operand staging: the tile (TI rows of the output dimension, BK of k) is
// read in pairs of consecutive doubles, along the output dimension for an
// "MN-major" operand (A not transposed, B transposed) or along k for a
// "K-major" one, and stored to LDS as [k][index].  An MN-major pair is one
// 16-byte LDS write (row pitch TI + 4, 16-byte aligned); a K-major pair is
// transposed on the way in with two 8-byte writes (odd pitch TI + 1, so that
// the lanes of a wavefront hit different banks).
template <bool KMAJ, int TI, int BK>
struct Stage {
    static constexpr int LD = KMAJ ? TI + 1 : TI + 4;
    static constexpr int PAIRS = TI * BK / 2;
    __device__ static __forceinline__ int idx(int c) { return KMAJ ? c / (BK / 2) : 2 * (c % (TI / 2)); }
    __device__ static __forceinline__ int kk(int c) { return KMAJ ? 2 * (c % (BK / 2)) : c / (TI / 2); }
    // memory offset (doubles) of element (index i, k) from the tile's origin
    __device__ static __forceinline__ long off(int i, int k, long ld) { return KMAJ ? k + (long)i * ld : i + (long)k * ld; }
    // the pair's second element
    __device__ static __forceinline__ int i2(int i) { return KMAJ ? i : i + 1; }
    __device__ static __forceinline__ int k2(int k) { return KMAJ ? k + 1 : k; }
};

// Tiles of the launch: every tile of C for a full product, the tiles on or
// below the diagonal for GEMM_LOWER; counted from the launch bounds M.host,
// N.host.  The grid is one-dimensional over exactly these tiles (blockIdx.y =
// split-K slice): the hardware deals workgroups to the 8 XCDs in turn, so a
// grid with idle tiles interleaved (the upper triangle) leaves the XCDs with
// unequal work, and in-order dispatch then stalls every XCD behind the
// busiest one.
template <int BM, int BN>
__host__ __device__ inline long tiles_of(const GemmArgs &p) {
    const long tm = (p.M.host + BM - 1) / BM, tn = (p.N.host + BN - 1) / BN;
    if (p.uplo != GEMM_LOWER) return tm * tn;
    // columns by = 0 .. tn-1 of the lower triangle hold tm - by tiles each (BM == BN)
    const long t = tn < tm ? tn : tm;
    return t * tm - t * (t - 1) / 2;
}

// Workgroup -> tile: the linear ids a single XCD receives (id mod 8) are
// given one contiguous run of the tile order, so that the workgroups resident
// on one XCD at a time share operand panels in its L2.  For a full product
// the order takes bands of TILE_BAND tile rows and walks each band column by
// column: a run of 32 consecutive tiles (one per compute unit of an XCD)
// covers 4 x 8 tiles and streams 4 panels of A and 8 of B, where a walk down
// whole columns of C streams 1 panel of B and 32 of A.  Bands of fewer rows
// at the bottom edge are walked the same way.
constexpr int TILE_BAND = 4;

template <int BM, int BN>
__device__ __forceinline__ void tile_of(const GemmArgs &p, int &bx, int &by) {
    const long T = gridDim.x;
    const long lin = blockIdx.x;
    const long q = T / 8, rem = T % 8, x = lin % 8;
    long t = x * q + (x < rem ? x : rem) + lin / 8;
    const int tm = (p.M.host + BM - 1) / BM;
    if (p.uplo != GEMM_LOWER) {
        const long tn = (p.N.host + BN - 1) / BN;
        const long band = t / (TILE_BAND * tn);
        const long in = t - band * TILE_BAND * tn;
        const int g = min(TILE_BAND, tm - (int)band * TILE_BAND);
        bx = (int)(band * TILE_BAND + in % g);
        by = (int)(in / g);
        return;
    }
    int c = 0;
    while (t >= tm - c) {
        t -= tm - c;
        ++c;
    }
    by = c;
    bx = c + (int)t;
}

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(WM * WN * 64) void dgemm_kernel(GemmArgs p) {
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    using SA = Stage<TA, BM, BK>;    // A stored K x M (k contiguous) when transposed
    using SB = Stage<!TB, BN, BK>;   // B stored K x N (k contiguous) when not transposed
    constexpr int LA = SA::LD, LB = SB::LD;
    constexpr int PA = SA::PAIRS / NT, PB = SB::PAIRS / NT;   // pairs per thread per chunk
    static_assert(PA * NT == SA::PAIRS && PB * NT == SB::PAIRS, "tile/thread mismatch");
    static_assert(TM % 16 == 0 && TN % 16 == 0 && BK % 4 == 0, "bad tile");

    __shared__ __align__(16) double As[2][BK][LA];
    __shared__ __align__(16) double Bs[2][BK][LB];

    const int M = p.M.get(), N = p.N.get(), K = p.K.get();
    int bx, by;
    tile_of<BM, BN>(p, bx, by);
    const int row0 = bx * BM, col0 = by * BN;
    if (row0 >= M || col0 >= N) return;

    int kbeg = 0, kend = K;
    double *C = p.C;
    if (p.splitk > 1) {
        const int chunk = (((K + p.splitk - 1) / p.splitk) + BK - 1) / BK * BK;
        kbeg = blockIdx.y * chunk;
        kend = min(K, kbeg + chunk);
        C += (long)blockIdx.y * p.strideC;
    }

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const double *__restrict__ A = p.A;
    const double *__restrict__ B = p.B;
    const long lda = p.lda, ldb = p.ldb;

    // Fast path (uniform): whole tile inside C, 16-byte aligned operands and
    // 32-bit offsets within a chunk.  Each thread's pair offsets relative to
    // the chunk origin are then computed once; a chunk only moves the
    // (scalar) origin.
    const bool aligned = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0 &&
                         ((lda | ldb) & 1) == 0;
    const bool small_off = (TA ? (long)BM * lda : (long)BK * lda) < (1L << 30) &&
                           (TB ? (long)BK * ldb : (long)BN * ldb) < (1L << 30);
    const bool interior = aligned && small_off && row0 + BM <= M && col0 + BN <= N;
    int aoff[PA], boff[PB], alds[PA], blds[PB];
#pragma unroll
    for (int q = 0; q < PA; ++q) {
        const int c = tid + NT * q;
        aoff[q] = (int)SA::off(SA::idx(c), SA::kk(c), lda);
        alds[q] = SA::kk(c) * LA + SA::idx(c);
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
        const int c = tid + NT * q;
        boff[q] = (int)SB::off(SB::idx(c), SB::kk(c), ldb);
        blds[q] = SB::kk(c) * LB + SB::idx(c);
    }

    d2 ra[PA], rb[PB];
    auto gload = [&](int kc) {
        if (interior && kc + BK <= kend) {
            const double *a0 = A + SA::off(row0, kc, lda);
            const double *b0 = B + SB::off(col0, kc, ldb);
#pragma unroll
            for (int q = 0; q < PA; ++q) ra[q] = *reinterpret_cast<const d2 *>(a0 + aoff[q]);
#pragma unroll
            for (int q = 0; q < PB; ++q) rb[q] = *reinterpret_cast<const d2 *>(b0 + boff[q]);
        } else {
#pragma unroll
            for (int q = 0; q < PA; ++q) {
                const int c = tid + NT * q;
                const int i = row0 + SA::idx(c), k = kc + SA::kk(c);
                ra[q].x = ld_or(A, SA::off(i, k, lda), i < M && k < kend, 0.0);
                ra[q].y = ld_or(A, SA::off(SA::i2(i), SA::k2(k), lda), SA::i2(i) < M && SA::k2(k) < kend, 0.0);
            }
#pragma unroll
            for (int q = 0; q < PB; ++q) {
                const int c = tid + NT * q;
                const int j = col0 + SB::idx(c), k = kc + SB::kk(c);
                rb[q].x = ld_or(B, SB::off(j, k, ldb), j < N && k < kend, 0.0);
                rb[q].y = ld_or(B, SB::off(SB::i2(j), SB::k2(k), ldb), SB::i2(j) < N && SB::k2(k) < kend, 0.0);
            }
        }
    };
    auto sstore = [&](int buf) {
        double *as = &As[buf][0][0];
        double *bs = &Bs[buf][0][0];
#pragma unroll
        for (int q = 0; q < PA; ++q) {
            if (TA) {
                as[alds[q]] = ra[q].x;
                as[alds[q] + LA] = ra[q].y;
            } else {
                *reinterpret_cast<d2 *>(as + alds[q]) = ra[q];
            }
        }
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            if (!TB) {
                bs[blds[q]] = rb[q].x;
                bs[blds[q] + LB] = rb[q].y;
            } else {
                *reinterpret_cast<d2 *>(bs + blds[q]) = rb[q];
            }
        }
    };

    static_assert(KFLUSH % BK == 0, "flush period must be whole chunks");
    constexpr int FLUSH_CHUNKS = KFLUSH / BK;
    d4 acc[FM][FN], tot[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            tot[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        }

    const int nchunks = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    if (nchunks > 0) {
        gload(kbeg);
        sstore(0);
        __syncthreads();
        for (int c = 0; c < nchunks; ++c) {
            const int buf = c & 1;
            const bool more = c + 1 < nchunks;
            if (more) gload(kbeg + (c + 1) * BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                double af[FM], bf[FN];
                const int kr = kk + (lane >> 4);
#pragma unroll
                for (int a = 0; a < FM; ++a) af[a] = As[buf][kr][wm * TM + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < FN; ++b) bf[b] = Bs[buf][kr][wn * TN + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
            }
            if ((c + 1) % FLUSH_CHUNKS == 0) {
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
                        tot[a][b] += acc[a][b];
                        acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
                    }
            }
            if (more) sstore(buf ^ 1);
            __syncthreads();
        }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) tot[a][b] += acc[a][b];

    const bool lower = p.uplo == GEMM_LOWER;
    const long ldc = p.ldc;
    const double alpha = p.alpha, beta = p.beta;
    const bool raw = p.splitk > 1;
    const bool with_c = !raw && beta != 0.0;   // uniform
    // the old values of C first, all in flight together, then the stores
    d4 cold[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
        const int r = row0 + wm * TM + a * 16 + (lane & 15);
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * TN + b * 16 + (lane >> 4) + 4 * v;
                cold[a][b][v] = ld_or(C, r + (long)c * ldc, with_c && r < M && c < N && (!lower || r >= c), 0.0);
            }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a) {
        const int r = row0 + wm * TM + a * 16 + (lane & 15);
#pragma unroll
        for (int b = 0; b < FN; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * TN + b * 16 + (lane >> 4) + 4 * v;
                if (r < M && c < N && (!lower || r >= c)) {
                    const double val = tot[a][b][v];
                    C[r + (long)c * ldc] = raw ? val : (with_c ? alpha * val + beta * cold[a][b][v] : alpha * val);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 128 x 128 tiles with direct global -> LDS operand loads
//
// Same tiling, tile order, two-level summation and epilogue as dgemm_kernel
// <128, 128, 32, 4, 2>, but the interior K chunks of interior tiles go from
// global memory straight into LDS (global_load_lds_dwordx4: no staging
// registers, no LDS store instructions, the next chunk in flight during the
// current one).  A wavefront's direct load fills 1 KiB of LDS, 16 bytes per
// lane in lane order, so the LDS layouts are:
//   MN-major operand (index contiguous in memory): [k][DM_LD] with a padded
//     row pitch; one k row (128 doubles) is one wavefront load.
//   K-major operand (k contiguous): [index][32], the 16 two-double granules
//     of row i XOR-permuted by i mod 16; four rows per load.  The matrix
//     cores read it a granule (k, k + 1) per lane, 16 consecutive rows at a
//     time, for two k steps at once: the LDS serves 16-byte reads 8 lanes at
//     a time in 128-byte bank rounds, which the permutation keeps distinct
//     (8-byte reads of one k would meet every bank twice).
// Edge tiles and the last partial K chunk are staged through registers into
// the same layouts.  The two stage buffers of each operand are separate LDS
// arrays and every read address is array + opaque per-lane offset +
// constant, so the compiler keeps reads of one buffer independent of the
// direct loads into the other.
// ---------------------------------------------------------------------------
constexpr int DM_T = 128, DM_BK = 32;
constexpr int DM_LD = DM_T + 4;   // MN-major LDS row pitch (doubles)

template <bool KMAJ>
struct DmOp {
    static constexpr int BYTES = KMAJ ? DM_T * DM_BK * 8 : DM_BK * DM_LD * 8;
    // LDS double index of element (index i, k)
    __device__ static __forceinline__ int lds_index(int i, int k) {
        return KMAJ ? i * DM_BK + (((k >> 1) ^ (i & 15)) << 1) + (k & 1) : k * DM_LD + i;
    }
};

template <bool TA, bool TB, int NW, bool FL>
__global__ __launch_bounds__(64 * NW) void dgemm_dma_kernel(GemmArgs p) {
    constexpr bool AK = TA, BK_ = !TB;   // K-major operands
    using OA = DmOp<AK>;
    using OB = DmOp<BK_>;
    // NW = 8: 4 x 2 wavefronts of 32 x 64; NW = 4: 2 x 2 wavefronts of 64 x 64
    static_assert(NW == 4 || NW == 8, "wavefronts per workgroup");
    constexpr int NT = 64 * NW, TM = NW == 8 ? 32 : 64, TN = 64, FM = TM / 16, FN = TN / 16;
    constexpr int WMW = DM_T / TM;                 // wavefronts along M
    constexpr int PIECES = 32 / NW;                // direct loads per operand per wavefront and chunk
    constexpr int PAIRS = DM_T * DM_BK / 2 / NT;   // staged pairs per operand per thread
    __shared__ __align__(1024) char As0[OA::BYTES];
    __shared__ __align__(1024) char As1[OA::BYTES];
    __shared__ __align__(1024) char Bs0[OB::BYTES];
    __shared__ __align__(1024) char Bs1[OB::BYTES];

    const int M = p.M.get(), N = p.N.get(), K = p.K.get();
    int bx, by;
    tile_of<DM_T, DM_T>(p, bx, by);
    const int row0 = bx * DM_T, col0 = by * DM_T;
    if (row0 >= M || col0 >= N) return;

    int kbeg = 0, kend = K;
    double *C = p.C;
    if (p.splitk > 1) {
        const int chunk = (((K + p.splitk - 1) / p.splitk) + DM_BK - 1) / DM_BK * DM_BK;
        kbeg = blockIdx.y * chunk;
        kend = min(K, kbeg + chunk);
        C += (long)blockIdx.y * p.strideC;
    }

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WMW, wn = wave / WMW;
    const double *__restrict__ A = p.A;
    const double *__restrict__ B = p.B;
    const long lda = p.lda, ldb = p.ldb;

    // interior tiles with 16-byte aligned operands take direct loads for
    // every whole chunk
    const bool aligned = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0 &&
                         ((lda | ldb) & 1) == 0;
    const bool small_off = 4L * (lda + ldb) + 64L * (lda + ldb) < (1L << 30);
    const bool interior = aligned && small_off && row0 + DM_T <= M && col0 + DM_T <= N;

    // ---- direct loads: per-lane element offsets (the same for the PIECES
    // loads of each operand a wavefront issues per chunk)
    //   MN-major: load q of wavefront w is k row w + NW q, lane l its granule l
    //   K-major: load q is rows 4 (w + NW q) .. +3, lane l row + l / 16, slot
    //            l % 16 holding granule (l % 16) ^ (row % 16) (4 NW q is a
    //            multiple of 16, so the row's residue is 4 (w % 4) + l / 16)
    auto dma_lane_off = [&](bool kmaj, long ld) -> int {
        if (!kmaj) return 2 * lane;
        const int r = lane >> 4;
        const int g = (lane & 15) ^ ((4 * (wave & 3) + r) & 15);
        return 2 * g + (int)(r * ld);
    };
    const int adl = dma_lane_off(AK, lda), bdl = dma_lane_off(BK_, ldb);
    // load q (0..PIECES-1) of each operand for the chunk at kc
    auto dma_piece = [&](int q, int kc, char *as, char *bs) {
        const int u = wave + NW * q;   // k row (MN-major) or row group (K-major)
        const double *ga = AK ? A + kc + (long)(row0 + 4 * u) * lda : A + row0 + (long)(kc + u) * lda;
        const double *gb = BK_ ? B + kc + (long)(col0 + 4 * u) * ldb : B + col0 + (long)(kc + u) * ldb;
        lds_load16(ga + adl, as + (AK ? u * 1024 : u * DM_LD * 8));
        lds_load16(gb + bdl, bs + (BK_ ? u * 1024 : u * DM_LD * 8));
    };
    auto dma = [&](int kc, char *as, char *bs) {
#pragma unroll
        for (int q = 0; q < PIECES; ++q) dma_piece(q, kc, as, bs);
    };

    // ---- staged fill (edge tiles, partial chunks), after the current chunk's
    // products so that it holds no registers across them: PAIRS pairs per
    // operand per thread, zero outside the operand, written to the same layouts
    auto pair_of = [&](bool kmaj, int q, int &i, int &k) {
        const int c = tid + NT * q;
        if (kmaj) { i = c / (DM_BK / 2); k = 2 * (c % (DM_BK / 2)); }
        else      { i = 2 * (c % (DM_T / 2)); k = c / (DM_T / 2); }
    };
    auto staged_fill = [&](int kc, char *as, char *bs) {
#pragma unroll
        for (int q = 0; q < PAIRS; ++q) {
            int i, k;
            d2 v;
            pair_of(AK, q, i, k);
            const int gi = row0 + i, gk = kc + k;
            if (AK) {
                v.x = ld_or(A, gk + (long)gi * lda, gi < M && gk < kend, 0.0);
                v.y = ld_or(A, gk + 1 + (long)gi * lda, gi < M && gk + 1 < kend, 0.0);
            } else {
                v.x = ld_or(A, gi + (long)gk * lda, gi < M && gk < kend, 0.0);
                v.y = ld_or(A, gi + 1 + (long)gk * lda, gi + 1 < M && gk < kend, 0.0);
            }
            *reinterpret_cast<d2 *>(as + 8 * OA::lds_index(i, k)) = v;
            pair_of(BK_, q, i, k);
            const int gj = col0 + i, gk2 = kc + k;
            if (BK_) {
                v.x = ld_or(B, gk2 + (long)gj * ldb, gj < N && gk2 < kend, 0.0);
                v.y = ld_or(B, gk2 + 1 + (long)gj * ldb, gj < N && gk2 + 1 < kend, 0.0);
            } else {
                v.x = ld_or(B, gj + (long)gk2 * ldb, gj < N && gk2 < kend, 0.0);
                v.y = ld_or(B, gj + 1 + (long)gk2 * ldb, gj + 1 < N && gk2 < kend, 0.0);
            }
            *reinterpret_cast<d2 *>(bs + 8 * OB::lds_index(i, k)) = v;
        }
    };

    // ---- matrix-core reads.  The chunk's 32 k go to the 8 k steps of the
    // 16 x 16 x 4 instruction as k = 8 (s / 2) + 2 (lane / 16) + s % 2 (any
    // assignment that both operands share sums the same products), so that
    // steps 2 t and 2 t + 1 of a K-major operand come from one granule.
    // Fragment a covers the wavefront's rows wm*TM + 16a + (lane % 16).
    // MN-major: one per-lane offset (k = 2 (lane / 16)) plus a constant per
    // step; K-major: one per-lane offset per step pair t (k = 8 t + 2 (lane / 16)).
    int aro[DM_BK / 8], bro[DM_BK / 8];
#pragma unroll
    for (int t = 0; t < DM_BK / 8; ++t) {
        const int k = 8 * t + 2 * (lane >> 4);
        aro[t] = 8 * OA::lds_index(lane & 15, k);
        bro[t] = 8 * OB::lds_index(lane & 15, k);
        if (!AK && t > 0) aro[t] = aro[0];
        if (!BK_ && t > 0) bro[t] = bro[0];
    }
#pragma unroll
    for (int t = 0; t < DM_BK / 8; ++t) {
        if (AK || t == 0) asm volatile("" : "+v"(aro[t]));
        if (BK_ || t == 0) asm volatile("" : "+v"(bro[t]));
    }
    // byte offset of row block r (a multiple of 16) at k step s, beyond the lane offset
    auto rconst = [&](bool kmaj, int r, int s) {
        return kmaj ? 8 * r * DM_BK : 8 * ((8 * (s / 2) + s % 2) * DM_LD + r);
    };

    constexpr int FLUSH_CHUNKS = KFLUSH / DM_BK;
    // FL: two-level sums (acc restarted every KFLUSH of K, totals in tot);
    // otherwise acc holds the whole sum
    d4 acc[FM][FN], tot[FL ? FM : 1][FL ? FN : 1];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            if constexpr (FL) tot[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        }
    // the products of one chunk; with `pf`, the direct loads of the next
    // chunk (at kn, into na / nb) are spread over its first k steps
    auto compute = [&](const char *as, const char *bs, bool pf, int kn, char *na, char *nb) {
#pragma unroll
        for (int t = 0; t < DM_BK / 8; ++t) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (2 * t + h < PIECES && pf) dma_piece(2 * t + h, kn, na, nb);
            double af[2][FM], bf[2][FN];
#pragma unroll
            for (int a = 0; a < FM; ++a) {
                if (AK) {
                    const d2 v = *reinterpret_cast<const d2 *>(as + aro[t] + rconst(true, wm * TM + a * 16, 0));
                    af[0][a] = v.x;
                    af[1][a] = v.y;
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        af[h][a] = *reinterpret_cast<const double *>(as + aro[0] +
                                                                      rconst(false, wm * TM + a * 16, 2 * t + h));
                }
            }
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                if (BK_) {
                    const d2 v = *reinterpret_cast<const d2 *>(bs + bro[t] + rconst(true, wn * TN + b * 16, 0));
                    bf[0][b] = v.x;
                    bf[1][b] = v.y;
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        bf[h][b] = *reinterpret_cast<const double *>(bs + bro[0] +
                                                                      rconst(false, wn * TN + b * 16, 2 * t + h));
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[h][b], af[h][a], acc[a][b], 0, 0, 0);
        }
    };

    const int nchunks = kend > kbeg ? (kend - kbeg + DM_BK - 1) / DM_BK : 0;
    auto direct = [&](int c) { return interior && kbeg + (c + 1) * DM_BK <= kend; };   // uniform
    // chunk c from buffer X while chunk c + 1 goes into buffer Y
    auto step = [&](int c, char *xa, char *xb, char *ya, char *yb) {
        const bool more = c + 1 < nchunks;
        const bool dnext = more && direct(c + 1);
        compute(xa, xb, dnext, kbeg + (c + 1) * DM_BK, ya, yb);
        if constexpr (FL) {
            if ((c + 1) % FLUSH_CHUNKS == 0) {
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
                        tot[a][b] += acc[a][b];
                        acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
                    }
            }
        }
        if (more && !dnext) staged_fill(kbeg + (c + 1) * DM_BK, ya, yb);
        wait_vm<0>();
        stage_barrier();
    };
    if (nchunks > 0) {
        if (direct(0)) dma(kbeg, As0, Bs0);
        else staged_fill(kbeg, As0, Bs0);
        wait_vm<0>();
        stage_barrier();
        int c = 0;
        for (; c + 1 < nchunks; c += 2) {
            step(c, As0, Bs0, As1, Bs1);
            step(c + 1, As1, Bs1, As0, Bs0);
        }
        if (c < nchunks) step(c, As0, Bs0, As1, Bs1);
    }
    if constexpr (FL) {
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) acc[a][b] += tot[a][b];
    }

    const bool lower = p.uplo == GEMM_LOWER;
    const long ldc = p.ldc;
    const double alpha = p.alpha, beta = p.beta;
    const bool raw = p.splitk > 1;
    const bool with_c = !raw && beta != 0.0;   // uniform
    d4 cold[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
        const int r = row0 + wm * TM + a * 16 + (lane & 15);
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * TN + b * 16 + (lane >> 4) + 4 * v;
                cold[a][b][v] = ld_or(C, r + (long)c * ldc, with_c && r < M && c < N && (!lower || r >= c), 0.0);
            }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a) {
        const int r = row0 + wm * TM + a * 16 + (lane & 15);
#pragma unroll
        for (int b = 0; b < FN; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * TN + b * 16 + (lane >> 4) + 4 * v;
                if (r < M && c < N && (!lower || r >= c)) {
                    const double val = acc[a][b][v];
                    C[r + (long)c * ldc] = raw ? val : (with_c ? alpha * val + beta * cold[a][b][v] : alpha * val);
                }
            }
        }
    }
}

template <bool TA, bool TB>
static hipError_t launch_dma_t(const GemmArgs &a, hipStream_t s) {
    const int S = a.splitk > 1 ? a.splitk : 1;
    const long T = tiles_of<DM_T, DM_T>(a);
    if (T <= 0) return hipSuccess;
    if (a.onelevel) hipLaunchKernelGGL((dgemm_dma_kernel<TA, TB, 8, false>), dim3((unsigned)T, S), dim3(512), 0, s, a);
    else hipLaunchKernelGGL((dgemm_dma_kernel<TA, TB, 8, true>), dim3((unsigned)T, S), dim3(512), 0, s, a);
    return hipGetLastError();
}

static hipError_t launch_dma(const GemmArgs &a, hipStream_t s) {
    if (a.transA) return a.transB ? launch_dma_t<true, true>(a, s) : launch_dma_t<true, false>(a, s);
    return a.transB ? launch_dma_t<false, true>(a, s) : launch_dma_t<false, false>(a, s);
}

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
static hipError_t launch_cfg_t(const GemmArgs &a, hipStream_t s) {
    static_assert(BM == BN, "square tiles (the lower-triangle walk assumes them)");
    const int S = a.splitk > 1 ? a.splitk : 1;
    const long T = tiles_of<BM, BN>(a);
    if (T <= 0) return hipSuccess;
    dim3 grid((unsigned)T, S);
    hipLaunchKernelGGL((dgemm_kernel<BM, BN, BK, WM, WN, TA, TB>), grid, dim3(WM * WN * 64), 0, s, a);
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN>
static hipError_t launch_cfg(const GemmArgs &a, hipStream_t s) {
    if (a.transA) return a.transB ? launch_cfg_t<BM, BN, BK, WM, WN, true, true>(a, s)
                                  : launch_cfg_t<BM, BN, BK, WM, WN, true, false>(a, s);
    return a.transB ? launch_cfg_t<BM, BN, BK, WM, WN, false, true>(a, s)
                    : launch_cfg_t<BM, BN, BK, WM, WN, false, false>(a, s);
}

// Split-K cost model for an output of `tiles` 128 x 128 tiles (one
// workgroup per compute unit at a time, so launches run in rounds of 256
// tiles) and depth K: the time is about rounds(S) x K / S chunk-steps plus the
// reduction of the S partial results, in microseconds.  Every split keeps at
// least 256 of K (a whole flush period of the two-level summation); S splits
// that leave less cost +infinity.
static double split_cost(long tiles, int K, int S) {
    const double chunk_us = 4.5;      // one 128 x 128 x 32 chunk of one workgroup
    const double reduce_us = 0.035;   // reading and adding one partial 128 x 128 tile
    const long kper = ((long)(K + S - 1) / S + 31) / 32 * 32;
    if (S > 1 && kper < 256) return __builtin_huge_val();
    const long rounds = (tiles * S + 255) / 256;
    return rounds * (kper / 32) * chunk_us + (S > 1 ? (S + 1) * tiles * reduce_us : 0.0);
}

// The cheapest split count up to maxS.  A small launch pays for its last,
// partly idle round; splitting K fills it.
int choose_splits(long tiles, int K, int maxS) {
    int best = 1;
    double bestc = 1e300;
    for (int S = 1; S <= maxS; ++S) {
        const double c = split_cost(tiles, K, S);
        if (c == __builtin_huge_val()) break;
        if (c < bestc * 0.98) {
            bestc = c;
            best = S;
        }
    }
    return best;
}

// The cheapest split count among those that give the 128 x 128 kernel at
// least 256 workgroups (tiles * S >= 256, S >= 2); 0 when there is none.
int fill_splits(long tiles, int K, int maxS) {
    const int smin = (int)std::max<long>(2, (255 + tiles) / tiles);
    int best = 0;
    double bestc = 1e300;
    for (int S = smin; S <= maxS; ++S) {
        const double c = split_cost(tiles, K, S);
        if (c == __builtin_huge_val()) break;
        if (c < bestc) {
            bestc = c;
            best = S;
        }
    }
    return best;
}

long gemm_tiles(const GemmArgs &a, int bm) {
    const long t = bm == 128 ? tiles_of<128, 128>(a) : tiles_of<64, 64>(a);
    return t * (a.splitk > 1 ? a.splitk : 1);
}

hipError_t launch_dgemm(const GemmArgs &a, hipStream_t s) {
    if (a.M.host <= 0 || a.N.host <= 0) return hipSuccess;
    // 128 x 128 tiles (8 wavefronts) when they alone fill the 256 compute
    // units; 64 x 64 tiles otherwise
    if (gemm_tiles(a, 128) >= 256 && a.K.host >= 128) return launch_dma(a, s);
    return launch_cfg<64, 64, 16, 2, 2>(a, s);
}

// ---------------------------------------------------------------------------
// split-K reduction: C = alpha * sum_z part[z] + beta * C
// ---------------------------------------------------------------------------
__global__ void splitk_reduce_kernel(const double *part, long ldp, long strideP, int S, double *C, long ldc,
                                     Dim Md, Dim Nd, double alpha, double beta, int uplo) {
    const int M = Md.get(), N = Nd.get();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= M || j >= N) return;
    if (uplo == GEMM_LOWER && i < j) return;
    double sum = 0.0;
    for (int z = 0; z < S; ++z) sum += part[z * strideP + i + (long)j * ldp];
    double *dst = C + i + (long)j * ldc;
    *dst = (beta != 0.0) ? alpha * sum + beta * (*dst) : alpha * sum;
}

hipError_t launch_splitk_reduce(const double *part, long ldp, long strideP, int S, double *C, long ldc, Dim M,
                                Dim N, double alpha, double beta, int uplo, hipStream_t s) {
    if (M.host <= 0 || N.host <= 0) return hipSuccess;
    dim3 grid((M.host + 255) / 256, N.host);
    hipLaunchKernelGGL(splitk_reduce_kernel, grid, dim3(256), 0, s, part, ldp, strideP, S, C, ldc, M, N, alpha,
                       beta, uplo);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fills and copies (no hipMemsetAsync: every step stays capturable in a graph)
// ---------------------------------------------------------------------------
__global__ void fill_kernel(double *X, long ldx, int rows, int cols, double v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < rows && j < cols) X[i + (long)j * ldx] = v;
}

hipError_t launch_fill(double *X, long ldx, int rows, int cols, double v, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    dim3 grid((rows + 255) / 256, cols);
    hipLaunchKernelGGL(fill_kernel, grid, dim3(256), 0, s, X, ldx, rows, cols, v);
    return hipGetLastError();
}

__global__ void fill_int_kernel(int *x, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

hipError_t launch_fill_int(int *x, int n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

__global__ void copy_kernel(const double *X, long ldx, double *Yp, long ldy, Dim Rd, Dim Cd) {
    const int rows = Rd.get(), cols = Cd.get();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < rows && j < cols) Yp[i + (long)j * ldy] = X[i + (long)j * ldx];
}

hipError_t launch_copy(const double *X, long ldx, double *Yp, long ldy, Dim rows, Dim cols, hipStream_t s) {
    if (rows.host <= 0 || cols.host <= 0) return hipSuccess;
    dim3 grid((rows.host + 255) / 256, cols.host);
    hipLaunchKernelGGL(copy_kernel, grid, dim3(256), 0, s, X, ldx, Yp, ldy, rows, cols);
    return hipGetLastError();
}

__global__ void axpby_kernel(const double *X, long ldx, double *Yp, long ldy, Dim Rd, Dim Cd, double a, double b) {
    const int rows = Rd.get(), cols = Cd.get();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < rows && j < cols) Yp[i + (long)j * ldy] = a * X[i + (long)j * ldx] + b * Yp[i + (long)j * ldy];
}

hipError_t launch_axpby(const double *X, long ldx, double *Yp, long ldy, Dim rows, Dim cols, double a, double b,
                        hipStream_t s) {
    if (rows.host <= 0 || cols.host <= 0) return hipSuccess;
    dim3 grid((rows.host + 255) / 256, cols.host);
    hipLaunchKernelGGL(axpby_kernel, grid, dim3(256), 0, s, X, ldx, Yp, ldy, rows, cols, a, b);
    return hipGetLastError();
}

// Upper triangle := transpose of the lower triangle, through 32 x 32 LDS tiles
// so that both the read and the write are column-contiguous.
__global__ void mirror_lower_kernel(double *X, long ldx, Dim nd) {
    __shared__ double t[32][33];
    const int n = nd.get();
    const int bi = blockIdx.x, bj = blockIdx.y;    // source tile (bi, bj) with bi >= bj
    if (bi < bj) return;
    const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = bi * 32 + tx, j = bj * 32 + ty + 8 * q;
        v[q] = ld_or(X, i + (long)j * ldx, i < n && j < n, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) t[ty + 8 * q][tx] = v[q];
    __syncthreads();
    // destination (j, i) for source (i, j) with i > j
    for (int yy = ty; yy < 32; yy += 8) {
        const int di = bj * 32 + tx;   // destination row = source column
        const int dj = bi * 32 + yy;   // destination column = source row
        if (di < n && dj < n && dj > di) X[di + (long)dj * ldx] = t[tx][yy];
    }
}

hipError_t launch_mirror_lower(double *X, long ldx, Dim n, hipStream_t s) {
    if (n.host <= 0) return hipSuccess;
    const int nt = (n.host + 31) / 32;
    hipLaunchKernelGGL(mirror_lower_kernel, dim3(nt, nt), dim3(32, 8), 0, s, X, ldx, n);
    return hipGetLastError();
}

}  // namespace geninv
