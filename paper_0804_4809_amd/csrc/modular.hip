// Int8 modular product engine of the mixed-precision form: the Gram matrix
// A = G'G (Section 2, Eq. (1)) and the chain's last product Y = P G'
// (Theorem 1) as exact products of fixed-point integer representations,
// evaluated on the int8 matrix cores of gfx950 (v_mfma_i32_16x16x64_i8).
//
// Representation: row i of op(A) gets the exponent ea_i (smallest e with
// max_k |op(A)_ik| < 2^e), column j of op(B) the exponent eb_j, and with a
// bit count beta, a_ik = rint(op(A)_ik 2^(beta - ea_i)) and
// b_kj = rint(op(B)_kj 2^(beta - eb_j)) are integers of magnitude <= 2^beta.
// The result is C_ij = 2^(ea_i + eb_j - 2 beta) sum_k a_ik b_kj with the
// integer sum exact and one final rounding to float64.
//
// Modular evaluation (the scheme of Ozaki, Uchino and Imamura, 2025): for N
// pairwise coprime moduli p_l <= 255 the residues a mod p_l, b mod p_l of
// magnitude <= 127 are int8 planes; one int8 GEMM per modulus sums at most
// 65536 products per launch slice (|sum| <= 65536 * 127^2 < 2^31, exact in
// int32), reduced mod p_l.  beta is chosen so that K 2^(2 beta) < M / 2
// (M = prod p_l), so the residues determine the signed sum, which is
// reconstructed by the Chinese remainder theorem in float64 pieces that are
// exact until the last two additions.  With N = 16 and K <= 2^17, beta = 52:
// the representation error is at most 2^-53 of each row/column maximum.
//
// Operands are K-contiguous int8 planes ("TN"): opA(i, k) = A_l[k + i lda],
// opB(k, j) = B_l[k + j ldb], the K extent zero-padded to a multiple of 64.
// The GEMM writes each modulus's residues (int8, summed over split-K slices
// by the reconstruction) in a tile-blocked layout that makes both the GEMM's
// stores and the reconstruction's loads 256-byte contiguous per wavefront:
// byte ((t NG + g) NT + thread) 4 + v for tile t, MFMA block g of the
// thread's NG blocks, accumulator slot v, NT threads per workgroup.
#include "common.h"

#include <cmath>

namespace geninv {

typedef int i4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// residues of the integer representation
// ---------------------------------------------------------------------------

// Residue planes are stored in 1 KiB blocks of 16 rows x 64 k, row group
// major (a row group's K extent is contiguous), each block already in the
// GEMM's LDS layout: granule g (16 k) of row r at slot g ^ mg_swz(r mod 16).
// A direct load of 16 rows of a stage is then one contiguous 1 KiB read
// (whole cache lines), not 64-byte halves of 16 lines.  The slot permutation
// makes the GEMM's 16-byte fragment reads (16 rows, one granule)
// bank-conflict free: the LDS serves them 8 (or 16) consecutive lanes at a
// time in bank rounds of 128 (or 256) bytes, which asks for distinct slots
// among rows of equal r mod 2 in each 8 (and of equal r mod 4 in each 16).
__host__ __device__ __forceinline__ int mg_swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// byte offset of element (row i, k) in a plane with ldp = Kpad bytes per row
__device__ __forceinline__ long mg_plane_off(long i, long k, long ldp) {
    return (i >> 4) * 16 * ldp + (k >> 6) * 1024 + (i & 15) * 64 + 16 * (((k & 63) >> 4) ^ mg_swz((int)(i & 15))) +
           (k & 15);
}

// x (an integer valued double, |x| <= 2^52) mod p, balanced to |r| <= p/2.
// q = rint(x / p) is within one of the nearest integer (x * (1/p) is off by
// less than |x| 2^-52 / p < 1), and x - q p is exact: one correction.
__device__ __forceinline__ int mod_balanced(double x, double p, double invp) {
    const double q = rint(x * invp);
    double r = fma(-q, p, x);
    const double h = 0.5 * p;
    r = r > h ? r - p : r;
    r = r < -h ? r + p : r;
    return (int)r;
}

// 16 residues (one byte each) of the representations of x[0..15] mod p,
// packed little-endian into four dwords
__device__ __forceinline__ uint4 residues16(const double (&v)[16], double p, double invp) {
    unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const unsigned b = (unsigned)(mod_balanced(v[q], p, invp) & 0xff);
        w[q >> 2] |= b << (8 * (q & 3));
    }
    return uint4{w[0], w[1], w[2], w[3]};
}

// plane l, element (j, k) = representation of X(k, j) mod p_l, column
// exponent e[j]; k = rows .. ldp-1 written as zeros.  A wavefront fills one
// plane block (16 columns j, 64 k) per modulus with one contiguous 1 KiB
// store: lane l takes column j0 + l / 4 and the 16 consecutive k of granule
// l % 4 (one 16-byte store per modulus).  A workgroup's four wavefronts take
// four consecutive k blocks.
__global__ __launch_bounds__(256) void mod_slice_cols_kernel(const double *X, long ldx, int rows, int cols,
                                                             const int *e, int beta, ModConsts mc, int8_t *planes,
                                                             long ldp, long sp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long k0 = ((long)blockIdx.y * 4 + wave) * 64 + 16 * (lane & 3);
    const int j = blockIdx.x * 16 + (lane >> 2);
    if (k0 >= ldp || j >= cols) return;
    const double *col = X + (long)j * ldx;
    const int sh = beta - e[j];
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = rint(ldexp(ld_or(col, k0 + q, k0 + q < rows, 0.0), sh));
    for (int l = 0; l < mc.n; ++l)
        *reinterpret_cast<uint4 *>(planes + l * sp + mg_plane_off(j, k0, ldp)) = residues16(v, mc.pf[l], mc.invp[l]);
}

// transposed: plane l, element (i, k) = representation of X(i, k) mod p_l,
// row exponent e[i]; k = cols .. ldp-1 zero.  A 64 x 64 (rows x k) tile of X is
// staged through LDS: read down the columns (64 rows = 512 contiguous bytes),
// then each thread takes 16 consecutive k of one row.
__global__ __launch_bounds__(256) void mod_slice_rows_t_kernel(const double *X, long ldx, int rows, int cols,
                                                               const int *e, int beta, ModConsts mc,
                                                               int8_t *planes, long ldp, long sp) {
    __shared__ double tile[64][65];
    const int i0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = i0 + tx, k = k0 + ty + 4 * q;
        tile[ty + 4 * q][tx] = ld_or(X, i + (long)k * ldx, i < rows && k < cols, 0.0);
    }
    __syncthreads();
    const int r = threadIdx.x >> 2, kc = (threadIdx.x & 3) * 16;
    const int i = i0 + r;
    const long k = k0 + kc;
    if (i >= rows || k >= ldp) return;
    const int sh = beta - e[i];
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = rint(ldexp(tile[kc + q][r], sh));
    for (int l = 0; l < mc.n; ++l)
        *reinterpret_cast<uint4 *>(planes + l * sp + mg_plane_off(i, k, ldp)) = residues16(v, mc.pf[l], mc.invp[l]);
}

// ---------------------------------------------------------------------------
// int8 GEMM per modulus
//
// A workgroup of WM x WN wavefronts owns a TILE x TILE tile of C for one
// modulus; a wavefront owns (TILE / WM) x (TILE / WN), FA x FB MFMA blocks of
// 16 x 16 (FA A fragments and FB B fragments per 64-deep stage feed FA FB
// matrix-core operations).  Two shapes: 128 x 128 with 2 x 2 wavefronts of
// 64 x 64 (three workgroups per compute unit), and 256 x 256 with 2 x 4
// wavefronts of 128 x 64 (one per compute unit), which halves the operand
// bytes each tile pulls from L2 per product (an int8 GEMM at the matrix
// cores' rate with 128 x 128 tiles would need about 39 TB/s of operands).
// K is taken 64 at a time: the stage's rows of 64 bytes (TILE A rows, then
// TILE B rows) go straight from global memory into LDS
// (global_load_lds_dwordx4, three buffers, loads two stages ahead).  A
// wavefront's direct load copies one 1 KiB plane block (16 rows, the
// stage's 64 k, granules already permuted by mg_swz) into a 1 KiB chunk.  Every fragment address
// is "buffer + opaque lane offset + constant", so the compiler keeps the
// three buffers apart in its wait counts.  The grid is one-dimensional over
// the tiles (lower triangle only for the Gram matrix), each XCD taking a
// contiguous run of an order that walks groups of MG_GM tile rows column by
// column; blockIdx.y is the split-K slice and blockIdx.z the modulus.
//
// Operand layout of v_mfma_i32_16x16x64_i8: lane l holds 16 int8 of row
// l % 16 (A) or column l % 16 (B), the same 16 k for A and B in both, so a
// fragment pair read with the same granule per lane sums over all 64 k of
// the stage.  The roles are swapped (the instruction gets the B rows as its
// A operand), so lane l holds C(row l % 16, column 4 (l / 16) + v).
// ---------------------------------------------------------------------------
constexpr int MG_BK = 64, MG_GM = 8;

constexpr int MG_MAX_STAGES = 1024;              // stages per split: sums of 65536 products

template <int TILE_, int WM_, int WN_>
struct MgCfg {
    static constexpr int TILE = TILE_, WM = WM_, WN = WN_;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int FA = TILE / WM / 16, FB = TILE / WN / 16;
    static constexpr int CHUNKS = 2 * TILE / 16;          // 1 KiB direct-load chunks per stage
    static constexpr int CPW = CHUNKS / (WM * WN);        // chunks per wavefront
    static constexpr int STAGE = 2 * TILE * MG_BK;        // LDS bytes per stage
    static constexpr int NG = FA * FB;                    // groups of 4 outputs per thread
    static_assert(CHUNKS % (WM * WN) == 0, "chunks per wavefront");
};
using MgSmall = MgCfg<128, 2, 2>;
using MgLarge = MgCfg<256, 2, 4>;

__host__ __device__ inline long mg_tiles(int M, int N, int lower, int tile) {
    const long tm = (M + tile - 1) / tile, tn = (N + tile - 1) / tile;
    if (!lower) return tm * tn;
    long t = 0;
    for (long r = 0; r < tm; ++r) t += r + 1 < tn ? r + 1 : tn;
    return t;
}

// logical tile t -> (bx, by): groups of MG_GM tile rows, column by column
__device__ inline void mg_tile(long t, int tm, int tn, int lower, int &bx, int &by) {
    int g0 = 0;
    for (;;) {
        const int g1 = min(g0 + MG_GM, tm);
        long cnt = 0;
        for (int r = g0; r < g1; ++r) cnt += lower ? min(r + 1, tn) : tn;
        if (t < cnt || g1 >= tm) break;
        t -= cnt;
        g0 = g1;
    }
    const int g1 = min(g0 + MG_GM, tm);
    for (int c = 0;; ++c) {
        const int lo = lower ? max(g0, c) : g0;
        const int nr = g1 - lo;
        if (t < nr) {
            bx = lo + (int)t;
            by = c;
            return;
        }
        t -= nr;
    }
}

template <class CF>
__global__ __launch_bounds__(CF::NT) void mod_gemm_kernel(ModGemmArgs p) {
    constexpr int TILE = CF::TILE, NT = CF::NT, FA = CF::FA, FB = CF::FB, CPW = CF::CPW, NWV = CF::WM * CF::WN;
    __shared__ __align__(1024) char Ls0[CF::STAGE];
    __shared__ __align__(1024) char Ls1[CF::STAGE];
    __shared__ __align__(1024) char Ls2[CF::STAGE];

    const int tm = (p.M + TILE - 1) / TILE, tn = (p.N + TILE - 1) / TILE;
    long tile;
    {
        // the hardware deals workgroups to the 8 XCDs in turn: give XCD x a
        // contiguous run of the tile order
        const long T = gridDim.x, lin = blockIdx.x;
        const long q = T / 8, rem = T % 8, x = lin % 8;
        tile = x * q + (x < rem ? x : rem) + lin / 8;
    }
    int bx = 0, by = 0;
    mg_tile(tile, tm, tn, p.lower, bx, by);
    const int row0 = bx * TILE, col0 = by * TILE;
    const int l = blockIdx.z;   // modulus
    const int nst_all = p.Kpad / MG_BK;
    const int per = (nst_all + p.splitk - 1) / p.splitk;
    const int st0 = blockIdx.y * per, st1 = min(nst_all, st0 + per);
    const int8_t *Ab = p.A + (long)l * p.sa;
    const int8_t *Bb = p.B + (long)l * p.sb;

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % CF::WM, wn = wave / CF::WM;

    // Direct loads: chunk q (16 rows; A rows for q < TILE / 16, B rows after)
    // is loaded by wavefront q % NWV: lane l copies bytes 16 l .. 16 l + 15 of
    // the plane block of the chunk's row group and the stage.  Row groups past
    // M (N) are read clamped: they only reach outputs that are never stored.
    constexpr int ACH = TILE / 16;
    unsigned srcoff[CPW];
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
        const int q = wave + NWV * i;
        const int grp = q < ACH ? min((row0 >> 4) + q % ACH, (p.M - 1) >> 4)
                                : min((col0 >> 4) + q % ACH, (p.N - 1) >> 4);
        srcoff[i] = (unsigned)((long)grp * 16 * (q < ACH ? p.lda : p.ldb) + 16 * lane);
    }
    auto dma = [&](int st, char *buf) {
        const long k0 = (long)st * 1024;   // the stage's block within a row group
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const int q = wave + NWV * i;
            lds_load16((q < ACH ? Ab : Bb) + k0 + srcoff[i], buf + q * 1024);
        }
    };

    i4 acc[FA][FB];
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] = i4{0, 0, 0, 0};

    // lane read offsets: row l % 16 of a 16-row block, granule l / 16
    constexpr int WTM = TILE / CF::WM, WTN = TILE / CF::WN;
    int rda = (wm * WTM + (lane & 15)) * 64 + 16 * ((lane >> 4) ^ mg_swz(lane & 15));
    int rdb = rda + (TILE + wn * WTN - wm * WTM) * 64;
    asm volatile("" : "+v"(rda), "+v"(rdb));
    auto compute = [&](const char *buf) {
        i4 bf[FB];
#pragma unroll
        for (int b = 0; b < FB; ++b) bf[b] = *reinterpret_cast<const i4 *>(buf + rdb + b * 16 * 64);
#pragma unroll
        for (int a = 0; a < FA; ++a) {
            const i4 af = *reinterpret_cast<const i4 *>(buf + rda + a * 16 * 64);
#pragma unroll
            for (int b = 0; b < FB; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(bf[b], af, acc[a][b], 0, 0, 0);
        }
    };
    auto stage = [&](int st, char *next, const char *cur) {
        dma(min(st + 2, st1 - 1), next);
        compute(cur);
        wait_vm<CPW>();    // this wavefront's loads of stage st + 1 landed
        stage_barrier();
    };
    if (st1 > st0) {
        dma(st0, Ls0);
        dma(min(st0 + 1, st1 - 1), Ls1);
        wait_vm<CPW>();
        stage_barrier();
        int st = st0;
        for (; st + 3 <= st1; st += 3) {
            stage(st, Ls2, Ls0);
            stage(st + 1, Ls0, Ls1);
            stage(st + 2, Ls1, Ls2);
        }
        if (st < st1) stage(st, Ls2, Ls0);
        if (st + 1 < st1) stage(st + 1, Ls0, Ls1);
        wait_vm<0>();
    }

    // residues, balanced: |acc| < 2^31 is exact in float64
    const double invp = p.mc.invp[l];
    const int pi = p.mc.p[l];
    unsigned *out = reinterpret_cast<unsigned *>(p.R + ((long)l * p.splitk + blockIdx.y) * p.strideR) +
                    (tile * CF::NG) * NT + tid;
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) {
            unsigned w = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int x = acc[a][b][v];
                const int q = (int)rint((double)x * invp);
                int r = x - q * pi;
                r = r > (pi >> 1) ? r - pi : r;
                r = r < -(pi >> 1) ? r + pi : r;
                w |= (unsigned)(r & 0xff) << (8 * v);
            }
            out[(a * FB + b) * NT] = w;
        }
}

// ---------------------------------------------------------------------------
// Chinese remainder reconstruction
//
// For one output: R_l = sum over split slices of the residues, s_l =
// (R_l y_l) mod p_l in [0, p_l) with y_l = (M / p_l)^-1 mod p_l, so that the
// signed integer sum X = sum_l s_l (M / p_l) - q M with q = rint(sum_l s_l /
// p_l) (|X| < M / 2 with a margin far above the float64 error of that sum).
// M / p_l and M are split into three float64 pieces on grids of 2^(E-40),
// 2^(E-80) and below (E = bit length of M): each piece has at most 40 (44)
// significant bits, so s_l times a piece is exact and so are the sums of the
// first two pieces over 16 moduli and the subtraction of q M; only the two
// final additions round (error about 2 u |X|).  Same tile and thread layout
// as the GEMM that wrote the residues.
// ---------------------------------------------------------------------------
template <class CF>
__global__ __launch_bounds__(CF::NT) void mod_reconstruct_kernel(ModRecArgs a) {
    constexpr int TILE = CF::TILE, NT = CF::NT, FB = CF::FB;
    constexpr int WTM = TILE / CF::WM, WTN = TILE / CF::WN;
    const long tile = blockIdx.x;
    const int tm = (a.M + TILE - 1) / TILE, tn = (a.N + TILE - 1) / TILE;
    int bx = 0, by = 0;
    mg_tile(tile, tm, tn, a.lower, bx, by);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % CF::WM, wn = wave / CF::WM;
    const int n = a.mc.n;
    for (int g = 0; g < CF::NG; ++g) {
        const int ba = g / FB, bb = g % FB;
        const int r = bx * TILE + wm * WTM + ba * 16 + (lane & 15);
        const int c0 = by * TILE + wn * WTN + bb * 16 + 4 * (lane >> 4);
        if (r >= a.M || c0 >= a.N || (a.lower && r < c0)) continue;
        double t[4] = {0, 0, 0, 0}, T1[4] = {0, 0, 0, 0}, T2[4] = {0, 0, 0, 0}, T3[4] = {0, 0, 0, 0};
        const long word = (tile * CF::NG + g) * NT + tid;
        // modulus l's residues of the 4 outputs: their sum over the K slices
        auto accumulate = [&](int l, const int (&R)[4]) {
            const int y = a.mc.y[l];
            const double pf = a.mc.pf[l], invp = a.mc.invp[l];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double x = (double)(R[v] * y);          // |R y| < 2^24: exact
                double s = fma(-floor(x * invp), pf, x);
                s = s < 0.0 ? s + pf : s;
                s = s >= pf ? s - pf : s;
                t[v] = fma(s, invp, t[v]);
                T1[v] = fma(s, a.mc.w1[l], T1[v]);
                T2[v] = fma(s, a.mc.w2[l], T2[v]);
                T3[v] = fma(s, a.mc.w3[l], T3[v]);
            }
        };
        if (a.splitk == 1) {
            // one residue word per modulus: all of them in flight at once
            unsigned wv[MOD_MAX];
#pragma unroll
            for (int l = 0; l < MOD_MAX; ++l)
                wv[l] = l < n ? reinterpret_cast<const unsigned *>(a.R + (long)l * a.strideR)[word] : 0u;
#pragma unroll
            for (int l = 0; l < MOD_MAX; ++l) {
                if (l >= n) break;
                int R[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) R[v] = (int)(signed char)((wv[l] >> (8 * v)) & 0xff);
                accumulate(l, R);
            }
        } else {
            for (int l = 0; l < n; ++l) {
                int R[4] = {0, 0, 0, 0};
                for (int z = 0; z < a.splitk; ++z) {
                    const unsigned w = reinterpret_cast<const unsigned *>(a.R + ((long)l * a.splitk + z) * a.strideR)[word];
#pragma unroll
                    for (int v = 0; v < 4; ++v) R[v] += (int)(signed char)((w >> (8 * v)) & 0xff);
                }
                accumulate(l, R);
            }
        }
        const int er = a.ea[r];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = c0 + v;
            if (c >= a.N || (a.lower && r < c)) continue;
            const double q = rint(t[v]);
            const double X = (fma(-q, a.mc.m1, T1[v]) + fma(-q, a.mc.m2, T2[v])) + fma(-q, a.mc.m3, T3[v]);
            a.C[r + (long)c * a.ldc] = ldexp(X, er + a.eb[c] - 2 * a.beta);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_mod_slice_cols(const double *X, long ldx, int rows, int cols, const int *e, int beta,
                                 const ModConsts &mc, int8_t *planes, long ldp, long sp, hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    if (ldp % 64 != 0 || sp % 16 != 0 || (reinterpret_cast<uintptr_t>(planes) & 15)) return hipErrorInvalidValue;
    dim3 grid((unsigned)((cols + 15) / 16), (unsigned)((ldp / 64 + 3) / 4));
    hipLaunchKernelGGL(mod_slice_cols_kernel, grid, dim3(256), 0, s, X, ldx, rows, cols, e, beta, mc, planes, ldp,
                       sp);
    return hipGetLastError();
}

hipError_t launch_mod_slice_rows_t(const double *X, long ldx, int rows, int cols, const int *e, int beta,
                                   const ModConsts &mc, int8_t *planes, long ldp, long sp, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (ldp % 64 != 0 || sp % 16 != 0 || (reinterpret_cast<uintptr_t>(planes) & 15)) return hipErrorInvalidValue;
    dim3 grid((rows + 63) / 64, (unsigned)(ldp / 64));
    hipLaunchKernelGGL(mod_slice_rows_t_kernel, grid, dim3(256), 0, s, X, ldx, rows, cols, e, beta, mc, planes,
                       ldp, sp);
    return hipGetLastError();
}

static int mg_tile_of(int cfg) { return cfg ? MgLarge::TILE : MgSmall::TILE; }

long mod_tiles(int M, int N, int lower, int cfg) { return mg_tiles(M, N, lower, mg_tile_of(cfg)); }

int mod_min_splits(int Kpad) { return (Kpad / MG_BK + MG_MAX_STAGES - 1) / MG_MAX_STAGES; }

size_t mod_residue_bytes(int M, int N, int lower, int cfg) {
    const long t = mg_tile_of(cfg);
    return (size_t)mg_tiles(M, N, lower, (int)t) * t * t;
}

hipError_t launch_mod_gemm(const ModGemmArgs &a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    if (a.Kpad % MG_BK != 0 || a.splitk < 1 || a.mc.n < 1 || a.mc.n > MOD_MAX) return hipErrorInvalidValue;
    const int nst = a.Kpad / MG_BK;
    if ((nst + a.splitk - 1) / a.splitk > MG_MAX_STAGES) return hipErrorInvalidValue;
    // lane offsets into a plane (row groups of 16 rows of lda bytes) are
    // 32-bit byte counts
    if ((double)((a.M + 15) / 16 * 16) * a.lda >= 4294967296.0 ||
        (double)((a.N + 15) / 16 * 16) * a.ldb >= 4294967296.0)
        return hipErrorInvalidValue;
    if ((size_t)a.strideR < mod_residue_bytes(a.M, a.N, a.lower, a.cfg)) return hipErrorInvalidValue;
    const long T = mod_tiles(a.M, a.N, a.lower, a.cfg);
    if (a.cfg)
        hipLaunchKernelGGL(mod_gemm_kernel<MgLarge>, dim3((unsigned)T, a.splitk, a.mc.n), dim3(MgLarge::NT), 0, s, a);
    else
        hipLaunchKernelGGL(mod_gemm_kernel<MgSmall>, dim3((unsigned)T, a.splitk, a.mc.n), dim3(MgSmall::NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mod_reconstruct(const ModRecArgs &a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    const long T = mod_tiles(a.M, a.N, a.lower, a.cfg);
    if (a.cfg)
        hipLaunchKernelGGL(mod_reconstruct_kernel<MgLarge>, dim3((unsigned)T), dim3(MgLarge::NT), 0, s, a);
    else
        hipLaunchKernelGGL(mod_reconstruct_kernel<MgSmall>, dim3((unsigned)T), dim3(MgSmall::NT), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host: moduli, reconstruction constants, bit count
// ---------------------------------------------------------------------------
namespace {
int gcd_i(int a, int b) {
    while (b) {
        const int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// inverse of a mod p (a, p coprime), extended Euclid
int inv_mod(long a, int p) {
    long t = 0, nt = 1, r = p, nr = ((a % p) + p) % p;
    while (nr) {
        const long q = r / nr;
        long tmp = t - q * nt;
        t = nt;
        nt = tmp;
        tmp = r - q * nr;
        r = nr;
        nr = tmp;
    }
    return (int)(t < 0 ? t + p : t);
}

typedef unsigned __int128 u128;

int bitlen(u128 x) {
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// the three float64 pieces of x on the grids 2^(E-40), 2^(E-80) and below
void split3(u128 x, int E, double &h, double &m, double &lo) {
    const int s1 = E - 40 > 0 ? E - 40 : 0, s2 = E - 80 > 0 ? E - 80 : 0;
    const u128 x1 = (x >> s1) << s1;
    const u128 r1 = x - x1;
    const u128 x2 = (r1 >> s2) << s2;
    const u128 x3 = r1 - x2;
    h = std::ldexp((double)(unsigned long long)(x1 >> s1), s1);
    m = std::ldexp((double)(unsigned long long)(x2 >> s2), s2);
    lo = (double)(unsigned long long)x3;
}
}  // namespace

// The N largest pairwise coprime integers <= 255 (greedy from 255 down) and
// the reconstruction constants; returns false for N outside 1..MOD_MAX.
bool mod_consts(int N, ModConsts &mc) {
    if (N < 1 || N > MOD_MAX) return false;
    int k = 0;
    for (int p = 255; p > 1 && k < N; --p) {
        bool ok = true;
        for (int i = 0; i < k; ++i) ok = ok && gcd_i(p, mc.p[i]) == 1;
        if (ok) mc.p[k++] = p;
    }
    if (k < N) return false;
    mc.n = N;
    u128 M = 1;
    for (int i = 0; i < N; ++i) M *= (u128)mc.p[i];
    const int E = bitlen(M);
    for (int i = 0; i < N; ++i) {
        const u128 W = M / (u128)mc.p[i];
        mc.y[i] = inv_mod((long)(W % (u128)mc.p[i]), mc.p[i]);
        mc.pf[i] = (double)mc.p[i];
        mc.invp[i] = 1.0 / (double)mc.p[i];
        split3(W, E, mc.w1[i], mc.w2[i], mc.w3[i]);
    }
    split3(M, E, mc.m1, mc.m2, mc.m3);
    mc.log2M = std::log2((double)M);
    return true;
}

// Largest beta <= 52 with 2 K 2^(2 beta) (1 + 2^-20) <= M; -1 if none.
int mod_beta(const ModConsts &mc, long K) {
    u128 M = 1;
    for (int i = 0; i < mc.n; ++i) M *= (u128)mc.p[i];
    if (K < 1) K = 1;
    int beta = -1;
    for (int b = 0; b <= 52; ++b) {
        if (2 * b + 1 + 64 - __builtin_clzll((unsigned long long)K) > 127) break;
        const u128 need = ((u128)(unsigned long long)K << (2 * b + 1));
        if (need + (need >> 20) <= M) beta = b;
    }
    return beta;
}

}  // namespace geninv
