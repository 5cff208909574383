// Error-free split products on the bfloat16 matrix cores of gfx950: the
// mixed-precision form of the Gram matrix A = G'G (Section 2, Eq. (1)) and of
// the chain's last product Y = P G' (Theorem 1).
//
// Operand slicing (the error-free transformation of Ozaki, Ogita, Oishi and
// Rump, Numer. Algorithms 2012): each row or column v of an operand gets an
// exponent e with max |v| < 2^e; v / 2^e in (-1, 1) is cut, most significant
// first, into `s` signed 8-bit integer slices by truncation toward zero.  A
// slice is an integer of magnitude <= 255, exact in bfloat16, and a product of
// two slices is an integer <= 255^2, exact in float32.
//
// Sliced product: C_ij = 2^(ea_i + eb_j) sum over every slice pair (t, u) of
// 2^(-8 (t+u+2)) (A_t B_u)_ij.  Every pair is needed: with all pairs the
// result is the exact product of the sliced operands, so a sliced Gram
// matrix is still the Gram matrix of a matrix (the representation of G) and
// keeps its (near) null space; a truncated pair set perturbs that null space
// to first order, which a rank-deficient G turns into a large error in G^+.
// The pairs of one weight class c = t + u share a float32 accumulator on
// v_mfma_f32_16x16x32_bf16; a class of p pairs stays an exactly represented
// integer (below 2^24) while p * 255^2 * k_span < 2^24; the kernel moves it
// into a float64 total (scaled by its class's exact power of two) every 192
// values of k for one pair, 96 for two and 64 for three or four.  Every
// integer product and class sum is therefore exact and only the float64
// totals round.
//
// Both operands are stored K-contiguous ("TN"): opA(i, k) = A_t[k + i lda],
// opB(k, j) = B_u[k + j ldb], planes `sa` / `sb` elements apart, with the K
// extent padded with zeros to a multiple of 64 by the slicing kernels.
#include "common.h"

#include <utility>

namespace geninv {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// exponents: smallest e with max |x| < 2^e, 0 for an all-zero vector
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bound_exponent(double mx) {
    if (!(mx > 0.0)) return 0;
    int p;
    (void)frexp(mx, &p);   // mx = f 2^p, f in [0.5, 1)
    return p;
}

__global__ __launch_bounds__(256) void col_exponent_kernel(const double *X, long ldx, int rows, int cols, int *e) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    if (j >= cols) return;
    double mx = 0.0;
    const double *col = X + (long)j * ldx;
    for (int i = threadIdx.x; i < rows; i += 256) mx = fmax(mx, fabs(col[i]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) e[j] = bound_exponent(red[0]);
}

// 64 rows per workgroup, four column groups of 64 threads: each wavefront
// reads 64 consecutive rows of every fourth column (512-byte segments)
__global__ __launch_bounds__(256) void row_exponent_kernel(const double *X, long ldx, int rows, int cols, int *e) {
    __shared__ double red[4][64];
    const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + r;
    double mx = 0.0;
    if (i < rows) {
        const double *row = X + i;
        int j = g;
        for (; j + 12 < cols; j += 16) {
            const double a0 = row[(long)j * ldx], a1 = row[(long)(j + 4) * ldx];
            const double a2 = row[(long)(j + 8) * ldx], a3 = row[(long)(j + 12) * ldx];
            mx = fmax(mx, fmax(fmax(fabs(a0), fabs(a1)), fmax(fabs(a2), fabs(a3))));
        }
        for (; j < cols; j += 4) mx = fmax(mx, fabs(row[(long)j * ldx]));
    }
    red[g][r] = mx;
    __syncthreads();
    if (g == 0 && i < rows) e[i] = bound_exponent(fmax(fmax(red[0][r], red[1][r]), fmax(red[2][r], red[3][r])));
}

// the s slices of x / 2^e, most significant first
template <int S>
__device__ __forceinline__ void slice_value(double x, int e, __bf16 *out) {
    double r = ldexp(x, -e);
#pragma unroll
    for (int t = 0; t < S; ++t) {
        r *= 256.0;
        const double st = trunc(r);
        r -= st;
        out[t] = (__bf16)(float)st;
    }
}

// eight consecutive slices t of one operand, packed for a 16-byte store
template <int S>
struct Slices8 {
    uint4 v[S];
};

template <int S>
__device__ __forceinline__ void slice8(const double (&x)[8], int e, Slices8<S> &out) {
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        __bf16 a[S], b[S];
        slice_value<S>(x[q], e, a);
        slice_value<S>(x[q + 1], e, b);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const unsigned lo = __builtin_bit_cast(unsigned short, a[t]);
            const unsigned hi = __builtin_bit_cast(unsigned short, b[t]);
            reinterpret_cast<unsigned *>(&out.v[t])[q / 2] = lo | (hi << 16);
        }
    }
}

// planes[t][i + j ldp] = slice t of X(i, j) with the column exponent e[j];
// rows rows..ldp-1 are written as zeros.  A thread takes 8 consecutive rows
// (one 16-byte store per slice); ldp is a multiple of 8.
template <int S>
__global__ __launch_bounds__(256) void slice_cols_kernel(const double *X, long ldx, int rows, int cols,
                                                         const int *e, __bf16 *planes, long ldp, long sp) {
    const long i0 = ((long)blockIdx.x * 256 + threadIdx.x) * 8;
    const int j = blockIdx.y;
    if (i0 >= ldp || j >= cols) return;
    const double *col = X + (long)j * ldx;
    double x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = ld_or(col, i0 + q, i0 + q < rows, 0.0);
    Slices8<S> o;
    slice8<S>(x, e[j], o);
#pragma unroll
    for (int t = 0; t < S; ++t) *reinterpret_cast<uint4 *>(planes + t * sp + i0 + (long)j * ldp) = o.v[t];
}

// transposed row slicing: planes[t][k + i ldp] = slice t of X(i, k) with the
// row exponent e[i]; k = cols..ldp-1 written as zeros (ldp a multiple of 8).
// A 32 x 64 (rows x k) tile is staged through LDS: read down the columns of
// X (32 rows = 256 contiguous bytes), written along its rows, each thread 8
// consecutive k of one row (one 16-byte store per slice).
template <int S>
__global__ __launch_bounds__(256) void slice_rows_t_kernel(const double *X, long ldx, int rows, int cols,
                                                           const int *e, __bf16 *planes, long ldp, long sp) {
    __shared__ double tile[64][33];
    const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int i = i0 + tx, k = k0 + ty + 8 * q;
        v[q] = ld_or(X, i + (long)k * ldx, i < rows && k < cols, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) tile[ty + 8 * q][tx] = v[q];
    __syncthreads();
    const int r = threadIdx.x >> 3, kc = (threadIdx.x & 7) * 8;   // row r of the tile, k0 + kc .. + 7
    const int i = i0 + r;
    const long k = k0 + kc;
    if (i >= rows || k >= ldp) return;
    double x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = tile[kc + q][r];
    Slices8<S> o;
    slice8<S>(x, e[i], o);
#pragma unroll
    for (int t = 0; t < S; ++t) *reinterpret_cast<uint4 *>(planes + t * sp + k + (long)i * ldp) = o.v[t];
}

// ---------------------------------------------------------------------------
// sliced GEMM
//
// A workgroup (8 wavefronts, 4 x 2) owns a 128 x 64 tile of C; a wavefront
// owns 32 x 32 (2 x 2 MFMA blocks).  K is taken 32 at a time: the 32-wide
// slab of every slice of both operands (S x 192 rows of 64 bytes) goes
// straight from global memory into LDS (global_load_lds_dwordx4, three
// buffers: the loads of stage st + 2 are in flight while stage st runs), and
// each wavefront then forms the slice pairs from its registers.
// Such a load writes 16 consecutive bytes per lane, a wavefront a 1 KiB
// chunk of 16 rows; the four 16-byte granules of row r sit in the chunk
// XOR-permuted by sg_swz(r), so that the operand reads (16 rows, one
// granule) meet distinct banks: the LDS serves 16-byte reads 8 (or 16)
// consecutive lanes at a time in bank rounds of 128 (or 256) bytes, which
// asks for distinct slots among the rows of equal r mod 2 in each 8 (and of
// equal r mod 4 in each 16); (r / 2 xor r / 4) mod 4 gives both.  The grid is one-dimensional over the needed
// tiles (lower triangle for the Gram matrix); each XCD takes a contiguous run
// of a tile order that walks groups of SG_GM tile rows column by column.
// ---------------------------------------------------------------------------
constexpr int SG_BM = 128, SG_BN = 64, SG_BK = 32;
__device__ __forceinline__ int sg_swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }
constexpr int SG_ROWS = SG_BM + SG_BN;    // LDS rows per slice per stage: A rows, then B rows
constexpr int SG_CHUNKS = SG_ROWS / 16;  // 1 KiB LDS chunks (16 rows of 64 bytes) per slice per stage
constexpr int SG_NT = 512;
constexpr int SG_GM = 8;                  // tile rows per group of the tile order

// tiles of a launch: all of C, or those meeting the lower triangle (row tile
// bx reaches column tiles by < 2 bx + 2, as BM = 2 BN)
__host__ __device__ inline long sg_tiles(int M, int N, int lower) {
    const long tm = (M + SG_BM - 1) / SG_BM, tn = (N + SG_BN - 1) / SG_BN;
    if (!lower) return tm * tn;
    long t = 0;
    for (long r = 0; r < tm; ++r) t += 2 * r + 2 < tn ? 2 * r + 2 : tn;
    return t;
}

// Weight class c = t + u of s-slice operands: its pair count, and the
// number of 32-deep stages after which its float32 sum is moved to float64.
// The sum stays an exact integer while pairs * 32 * stages * 255^2 < 2^24;
// the kernel runs in cycles of 6 stages (its 3 LDS buffers twice over) and
// flushes one pair every 6 stages, two pairs every 3 and three or four pairs
// every 2.  Every class is also flushed at the end of a range.
constexpr int SG_CYCLE = 6;
__host__ __device__ constexpr int sg_pairs(int S, int c) {
    return (c < S ? c + 1 : 2 * S - 1 - c);
}
__host__ __device__ constexpr int sg_period(int S, int c) {
    return sg_pairs(S, c) == 1 ? 6 : (sg_pairs(S, c) == 2 ? 3 : 2);
}
static_assert(1 * 32 * 6 * 255 * 255 < (1 << 24) && 2 * 32 * 3 * 255 * 255 < (1 << 24) &&
                  4 * 32 * 2 * 255 * 255 < (1 << 24),
              "class periods must keep float32 class sums exact");

template <int S, int NC, int C>
__device__ __forceinline__ void sg_flush_class(f4 (&acc)[NC][2][2], double (&tot)[2][2][4]) {
    const double w = __builtin_bit_cast(double, (unsigned long long)(1023 - 8 * (C + 2)) << 52);   // 2^(-8 (C+2))
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) tot[a][b][v] = fma(w, (double)acc[C][a][b][v], tot[a][b][v]);
            acc[C][a][b] = f4{0.f, 0.f, 0.f, 0.f};
        }
}

// after stage J of a run (or every class when `all`)
template <int S, int NC, int J, int... C>
__device__ __forceinline__ void sg_flush_due(std::integer_sequence<int, C...>, bool all, f4 (&acc)[NC][2][2],
                                             double (&tot)[2][2][4]) {
    ((((J + 1) % sg_period(S, C) == 0 || all) ? sg_flush_class<S, NC, C>(acc, tot) : void()), ...);
}

// S slices per operand; the pairs of the NC weight classes t + u < NC
template <int S, int NC>
__global__ __launch_bounds__(SG_NT) void sliced_gemm_kernel(SlicedGemmArgs p) {
    static_assert(NC >= 1 && NC <= 2 * S - 1, "class count");
    // three stage buffers (loads run two stages ahead), separate arrays so
    // that reads of one need not wait for the direct loads into another
    __shared__ __align__(1024) char Ls0[S * SG_ROWS * 64];
    __shared__ __align__(1024) char Ls1[S * SG_ROWS * 64];
    __shared__ __align__(1024) char Ls2[S * SG_ROWS * 64];

    // workgroup -> tile: each XCD gets a contiguous run of the tile order, and
    // the order walks groups of SG_GM tile rows, column by column inside a
    // group, so that the ~32 tiles resident on one XCD form a block of about
    // SG_GM x 4 tiles sharing their operand panels in its L2
    const int tm = (p.M + SG_BM - 1) / SG_BM;
    const int tn = (p.N + SG_BN - 1) / SG_BN;
    int bx = 0, by = 0;
    {
        const long T = gridDim.x, lin = blockIdx.x;
        const long q = T / 8, rem = T % 8, x = lin % 8;
        long t = x * q + (x < rem ? x : rem) + lin / 8;
        int g0 = 0;
        for (;;) {   // the group holding tile t
            const int g1 = min(g0 + SG_GM, tm);
            long cnt = 0;
            for (int r = g0; r < g1; ++r) cnt += p.lower ? min(2 * r + 2, tn) : tn;
            if (t < cnt) break;
            t -= cnt;
            g0 = g1;
        }
        const int g1 = min(g0 + SG_GM, tm);
        for (int c = 0;; ++c) {   // column c of the group: rows reaching it
            const int lo = p.lower ? max(g0, c / 2) : g0;
            const int rows = g1 - lo;
            if (t < rows) {
                bx = lo + (int)t;
                by = c;
                break;
            }
            t -= rows;
        }
    }
    const int row0 = bx * SG_BM, col0 = by * SG_BN;

    const int nst_all = p.Kpad / SG_BK;
    int st0 = 0, st1 = nst_all;
    double *C = p.C;
    if (p.splitk > 1) {
        const int per = (nst_all + p.splitk - 1) / p.splitk;
        st0 = blockIdx.y * per;
        st1 = min(nst_all, st0 + per);
        C += (long)blockIdx.y * p.strideC;
    }

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 3, wn = wave >> 2;

    // Direct loads of a stage: chunk q (slice q / 12; A rows for the first 8
    // chunks of a slice, B rows for the last 4) is loaded by wavefront q % 8.
    // Lane l fills row l / 4 of its chunk, slot l % 4, with granule
    // (l % 4) ^ sg_swz(l / 4).  Rows past M (N) are read clamped: they only reach
    // rows (columns) of C that are never stored.
    constexpr int NCH = S * SG_CHUNKS;
    constexpr int CPW = (NCH + 7) / 8;   // chunks per wavefront
    // per chunk: a uniform base (operand and slice) and this lane's element
    // offset inside the slice plane (below 2^32: planes hold < 2^32 elements)
    unsigned srcoff[CPW];
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
        const int q = wave + 8 * i < NCH ? wave + 8 * i : wave;
        const int cq = q % SG_CHUNKS;
        const int r = (cq % 8) * 16 + (lane >> 2);
        const int g = (lane & 3) ^ sg_swz(lane >> 2);
        srcoff[i] = cq < 8 ? (unsigned)((long)min(row0 + r, p.M - 1) * p.lda + 8 * g)
                           : (unsigned)((long)min(col0 + r, p.N - 1) * p.ldb + 8 * g);
    }
    auto chunk_base = [&](int i) {
        const int q = wave + 8 * i < NCH ? wave + 8 * i : wave;
        const int t = q / SG_CHUNKS, cq = q % SG_CHUNKS;
        return cq < 8 ? p.A + (long)t * p.sa : p.B + (long)t * p.sb;
    };
    auto dma = [&](int st, char *buf) {
        const long k0 = (long)st * SG_BK;
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            // a wavefront without an i-th chunk reloads its first one (same
            // bytes to the same place), so every wavefront issues CPW loads
            const int q = NCH % 8 == 0 || wave + 8 * i < NCH ? wave + 8 * i : wave;
            lds_load16(chunk_base(i) + k0 + srcoff[i], buf + q * 1024);
        }
    };

    f4 acc[NC][2][2];
    double tot[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c][a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) tot[a][b][v] = 0.0;
        }

    // stage st from LDS buffer B: every slice pair, A slices one at a time
    // (all B slices held), into the pair's weight class
    // Per-lane LDS read offsets of the wavefront's A and B blocks (lane l:
    // row l % 16 of a 16-row block, granule l / 16), computed once and kept
    // opaque, so that every fragment address is one array plus this offset
    // plus a constant: the compiler then still sees which stage buffer a read
    // touches, and does not make it wait for loads into the other buffers.
    int rda = (wm * 32 + (lane & 15)) * 64 + 16 * ((lane >> 4) ^ sg_swz(lane & 15));
    int rdb = rda + (SG_BM + wn * 32 - wm * 32) * 64;
    asm volatile("" : "+v"(rda), "+v"(rdb));
    auto compute = [&](const char *buf) {
        bf8 bfr[S][2];
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                bfr[u][b] = *reinterpret_cast<const bf8 *>(buf + rdb + (u * SG_ROWS + b * 16) * 64);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            bf8 af[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                af[a] = *reinterpret_cast<const bf8 *>(buf + rda + (t * SG_ROWS + a * 16) * 64);
#pragma unroll
            for (int u = 0; u < S; ++u) {
                if (t + u >= NC) continue;
                const int c = t + u < NC ? t + u : 0;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[c][a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[u][b], af[a], acc[c][a][b], 0, 0, 0);
            }
        }
    };
    // Stage st: start the loads of stage st + 2 (clamped to the last stage of
    // the range: the extra loads land in a buffer no later stage reads),
    // compute stage st, flush the classes whose period ends, wait until this
    // wavefront's loads of stage st + 1 have landed (those of st + 2 may stay
    // in flight), barrier.  Full cycles of 6 stages run with their buffers and
    // flushes fixed at compile time; the last nst % 6 stages flush every class.
    auto buf_of = [&](auto bc) -> char * {
        constexpr int b = decltype(bc)::value;
        if constexpr (b == 0) return Ls0;
        else if constexpr (b == 1) return Ls1;
        else return Ls2;
    };
    // wait until only the latest stage's loads of this wavefront are pending
    auto wait_prev = [&]() { wait_vm<CPW>(); };
    const auto all_classes = std::make_integer_sequence<int, NC>{};
    auto stage = [&](int st, auto jc) {
        constexpr int J = decltype(jc)::value;
        dma(min(st + 2, st1 - 1), buf_of(std::integral_constant<int, (J + 2) % 3>{}));
        compute(buf_of(std::integral_constant<int, J % 3>{}));
        sg_flush_due<S, NC, J>(all_classes, false, acc, tot);
        wait_prev();
        stage_barrier();
    };
    if (st1 > st0) {
        dma(st0, Ls0);
        dma(min(st0 + 1, st1 - 1), Ls1);
        wait_prev();   // stage st0 landed
        stage_barrier();
        const int ncyc = (st1 - st0) / SG_CYCLE;
        int st = st0;
        for (int c = 0; c < ncyc; ++c, st += SG_CYCLE) {
            stage(st, std::integral_constant<int, 0>{});
            stage(st + 1, std::integral_constant<int, 1>{});
            stage(st + 2, std::integral_constant<int, 2>{});
            stage(st + 3, std::integral_constant<int, 3>{});
            stage(st + 4, std::integral_constant<int, 4>{});
            stage(st + 5, std::integral_constant<int, 5>{});
        }
        for (int i = 0; st < st1; ++i, ++st) {   // buffer of stage st: i mod 3
            const int bi = i % 3, bn = (i + 2) % 3;
            dma(min(st + 2, st1 - 1), bn == 0 ? Ls0 : (bn == 1 ? Ls1 : Ls2));
            compute(bi == 0 ? Ls0 : (bi == 1 ? Ls1 : Ls2));
            sg_flush_due<S, NC, 0>(all_classes, true, acc, tot);
            wait_prev();
            stage_barrier();
        }
        wait_vm<0>();
    }

    // result element (row, col): MFMA row index = column of C (4 (lane/16) + v),
    // MFMA column index = row of C (lane & 15)
    const bool raw = p.splitk > 1;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int r = row0 + wm * 32 + a * 16 + (lane & 15);
        if (r >= p.M) continue;
        const int er = p.ea[r];
        double old[2][4];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * 32 + b * 16 + 4 * (lane >> 4) + v;
                old[b][v] = ld_or(C, r + (long)c * p.ldc,
                                  !raw && p.beta != 0.0 && c < p.N && !(p.lower && r < c), 0.0);
            }
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * 32 + b * 16 + 4 * (lane >> 4) + v;
                if (c >= p.N || (p.lower && r < c)) continue;
                const double val = ldexp(tot[a][b][v], er + p.eb[c]);
                C[r + (long)c * p.ldc] = raw ? val : ((p.beta != 0.0) ? val + p.beta * old[b][v] : val);
            }
    }
}

hipError_t launch_col_exponents(const double *X, long ldx, int rows, int cols, int *e, hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_exponent_kernel, dim3(cols), dim3(256), 0, s, X, ldx, rows, cols, e);
    return hipGetLastError();
}

hipError_t launch_row_exponents(const double *X, long ldx, int rows, int cols, int *e, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(row_exponent_kernel, dim3((rows + 63) / 64), dim3(256), 0, s, X, ldx, rows, cols, e);
    return hipGetLastError();
}

template <int S>
static hipError_t slice_cols_s(const double *X, long ldx, int rows, int cols, const int *e, __bf16 *planes, long ldp,
                               long sp, hipStream_t s) {
    dim3 grid((ldp / 8 + 255) / 256, cols);
    hipLaunchKernelGGL((slice_cols_kernel<S>), grid, dim3(256), 0, s, X, ldx, rows, cols, e, planes, ldp, sp);
    return hipGetLastError();
}

template <int S>
static hipError_t slice_rows_t_s(const double *X, long ldx, int rows, int cols, const int *e, __bf16 *planes,
                                 long ldp, long sp, hipStream_t s) {
    dim3 grid((rows + 31) / 32, (ldp + 63) / 64);
    hipLaunchKernelGGL((slice_rows_t_kernel<S>), grid, dim3(256), 0, s, X, ldx, rows, cols, e, planes, ldp, sp);
    return hipGetLastError();
}

hipError_t launch_slice_cols(const double *X, long ldx, int rows, int cols, const int *e, int nslices,
                             __bf16 *planes, long ldp, long sp, hipStream_t s) {
    if (rows < 0 || cols <= 0) return hipSuccess;
    if (ldp % 8 != 0 || sp % 8 != 0 || (reinterpret_cast<uintptr_t>(planes) & 15)) return hipErrorInvalidValue;
    switch (nslices) {
        case 1: return slice_cols_s<1>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 2: return slice_cols_s<2>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 3: return slice_cols_s<3>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 4: return slice_cols_s<4>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 5: return slice_cols_s<5>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 6: return slice_cols_s<6>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_slice_rows_t(const double *X, long ldx, int rows, int cols, const int *e, int nslices,
                               __bf16 *planes, long ldp, long sp, hipStream_t s) {
    if (rows <= 0 || cols < 0) return hipSuccess;
    if (ldp % 8 != 0 || sp % 8 != 0 || (reinterpret_cast<uintptr_t>(planes) & 15)) return hipErrorInvalidValue;
    switch (nslices) {
        case 1: return slice_rows_t_s<1>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 2: return slice_rows_t_s<2>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 3: return slice_rows_t_s<3>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 4: return slice_rows_t_s<4>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 5: return slice_rows_t_s<5>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 6: return slice_rows_t_s<6>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        default: return hipErrorInvalidValue;
    }
}

template <int S, int NC>
static hipError_t launch_sliced_s(const SlicedGemmArgs &a, hipStream_t s) {
    const long T = sg_tiles(a.M, a.N, a.lower);
    const int Z = a.splitk > 1 ? a.splitk : 1;
    hipLaunchKernelGGL((sliced_gemm_kernel<S, NC>), dim3((unsigned)T, Z), dim3(SG_NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sliced_gemm(const SlicedGemmArgs &a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    if (a.Kpad % 64 != 0) return hipErrorInvalidValue;
    // lane offsets into a slice plane are 32-bit element counts
    if ((double)(a.M - 1) * a.lda + a.Kpad >= 4294967296.0 || (double)(a.N - 1) * a.ldb + a.Kpad >= 4294967296.0)
        return hipErrorInvalidValue;
    // every pair, or the pairs of weight at least 2^(-8 (S + 2)) (t + u <= S)
    const bool all = a.nclass == 2 * a.S - 1;
    if (!all && a.nclass != sliced_chain_classes(a.S)) return hipErrorInvalidValue;
    switch (a.S) {
        case 1: return launch_sliced_s<1, 1>(a, s);
        case 2: return launch_sliced_s<2, 3>(a, s);
        case 3: return all ? launch_sliced_s<3, 5>(a, s) : launch_sliced_s<3, 4>(a, s);
        case 4: return all ? launch_sliced_s<4, 7>(a, s) : launch_sliced_s<4, 5>(a, s);
        default: return hipErrorInvalidValue;
    }
}

long sliced_tiles(int M, int N, int lower) { return sg_tiles(M, N, lower); }

}  // namespace geninv
