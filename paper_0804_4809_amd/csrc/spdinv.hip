// M = (L'L)^-1 (Theorem 1) on gfx950 by block Gauss-Jordan elimination in
// its symmetric form (the sweep operator).
//
// L'L is symmetric positive definite (L has full column rank r), so every
// pivot block met by the elimination without pivoting is a Schur complement
// of an SPD matrix and is itself SPD.  One sweep of pivot block b (GJ_NB
// wide) of the r x r matrix B is
//
//   D       = B_bb^-1                        (pivot block, inverted in LDS)
//   R_j     = D B_bj          for j != b      (new pivot block row)
//   B_ij   -= B_ib R_j        for i, j != b   (rank-GJ_NB update)
//   B_ib    = B_ib D          for i != b      (new pivot block column, = R_i')
//   B_bj    = R_j,  B_bb = -D
//
// Every sweep keeps B symmetric, so only the blocks on or below the block
// diagonal are computed (diagonal blocks in full), half the update's work
// and traffic; after the last sweep B holds -B^-1, which the finishing
// kernel negates and mirrors.  Two launches per sweep: the panel kernel (D,
// R and a copy of the old block column, one workgroup per block column) and
// the update kernel (one workgroup per 64 x 64 tile), which reads only the
// staged panels so that tiles can be rewritten in place.  The 64 x 64 x 64
// tile products run on v_mfma_f64_16x16x4f64.  The rank r is read from
// device memory; steps and tiles past r exit at once.
#include "common.h"

#include <utility>

namespace geninv {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GJ_LD = GJ_NB + 1;

// Tile product on the matrix cores: the 64 x 64 result of Xs * Ys, where
// Xs[k][i] holds the left factor's column k and Ys[j][k] the right factor's
// column j (K = 64, zero padded).  Wavefront w owns rows 32 (w & 1) .. +31 and
// columns 32 (w >> 1) .. +31 as 2 x 2 blocks of 16 x 16; result element
// (row, col) is acc[a][b][v] with row = 32 (w & 1) + 16 a + (lane & 15) and
// col = 32 (w >> 1) + 16 b + (lane >> 4) + 4 v.
__device__ __forceinline__ void tile64_mfma(const double (*Xs)[GJ_LD], const double (*Ys)[GJ_LD], d4 acc[2][2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < GJ_NB; kk += 4) {
        const int kr = kk + (lane >> 4);
        double af[2], bf[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = Xs[kr][wm * 32 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; ++b) bf[b] = Ys[wn * 32 + b * 16 + (lane & 15)][kr];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
    }
}

// 1 / x for a positive normal x: the hardware estimate refined by two Newton
// steps (within an ulp or so of the correctly rounded quotient, and a much
// shorter dependency chain than the IEEE division sequence)
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
    return y;
}

// Gauss-Jordan inverse of the SPD block held in X (column-major X[j][i]),
// w x w in the top-left corner and identity elsewhere.  The 256 threads form
// a 16 x 16 grid of 4 x 4 sub-blocks: thread t keeps rows 4 rb .. 4 rb + 3 and
// columns 4 cb .. 4 cb + 3 (rb = t mod 16, cb = t / 16) in registers for the
// whole elimination.  A step eliminates the pivot pair P = {p, p + 1} (p
// even) at once, the 2 x 2 block form of the scalar steps: with E =
// X(P, P)^-1 (X(P, P) is a Schur complement of an SPD matrix, so symmetric
// positive definite, and E comes from its determinant),
//   X(i, j) -= X(i, P) E X(P, j)   (i, j not in P),   X(P, j) = E X(P, j),
//   X(i, P) = -X(i, P) E,                              X(P, P) = E.
// The two pivot rows and columns are published through LDS, double buffered
// by the parity of p / 2 (a buffer is rewritten two steps later, after every
// thread has passed the barrier of the step in between), so one barrier per
// pair of pivots suffices.  A step's cost is mostly the instruction issue of
// one wavefront per SIMD plus the barrier, LDS round trip and reciprocal on
// its dependency chain; per pivot the pair form issues about a fifth fewer
// instructions and has half as many of the latter.  For odd w
// the last pair takes pivot w from the identity padding: its row and column
// are zero off the diagonal, so the step reduces to the scalar one and the
// padding stays zero next to the w x w block.  On return X holds the
// inverse.  Returns false (uniformly) if a pivot is not positive.
template <int P>
__device__ __forceinline__ void gj_publish2(const double (&v)[4][4], int rb, int cb, double (*colb)[2][4][16],
                                            double (*rowb)[2][4][16]) {
    constexpr int b = (P >> 1) & 1, pq = P >> 2, pr = P & 3;
    if (cb == pq) {
        // row 4 rb + i of column p + k at [k][i][rb] (so that no two of a
        // thread's stores are adjacent and none needs its values gathered
        // into consecutive registers)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            colb[b][0][i][rb] = v[i][pr];       // column p
            colb[b][1][i][rb] = v[i][pr + 1];   // column p + 1
        }
    }
    if (rb == pq) {
        // column 4 cb + j of row p + k at [k][j][cb]
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            rowb[b][0][j][cb] = v[pr][j];       // row p
            rowb[b][1][j][cb] = v[pr + 1][j];   // row p + 1
        }
    }
}

// Every entry takes one form, y = x m + W0_i R0_j + W1_i R1_j: away from
// the pivots m = 1, W_i = -X(i, P) E (the new pivot column's values) and
// R_j = X(P, j), the rank-two update.  On the thread's pivot rows (prow) W_i
// is the row of E and m = 0, which gives E X(P, j); on its pivot columns
// (pcol) R_j is the column of the identity and m = 0, which gives -X(i, P) E,
// and both together give E.
template <int PR, int I, int J>
__device__ __forceinline__ void gj_entry2(double &x, const double (&W0)[4], const double (&W1)[4],
                                          const double (&R0)[4], const double (&R1)[4], double mr, double mc,
                                          double mrc) {
    constexpr bool pi = I == PR || I == PR + 1, pj = J == PR || J == PR + 1;
    const double xm = pi && pj ? x * mrc : pi ? x * mr : pj ? x * mc : x;
    x = __builtin_fma(W0[I], R0[J], __builtin_fma(W1[I], R1[J], xm));
}

template <int PR, int... E>
__device__ __forceinline__ void gj_entries2(std::integer_sequence<int, E...>, double (&v)[4][4],
                                            const double (&W0)[4], const double (&W1)[4], const double (&R0)[4],
                                            const double (&R1)[4], double mr, double mc, double mrc) {
    (gj_entry2<PR, (E >> 2), (E & 3)>(v[E >> 2][E & 3], W0, W1, R0, R1, mr, mc, mrc), ...);
}

template <int S>
__device__ __forceinline__ void gj_step2(double (&v)[4][4], bool &ok, int w, int rb, int cb,
                                         double (*colb)[2][4][16], double (*rowb)[2][4][16]) {
    constexpr int P = 2 * S;
    if (P >= w) return;   // identity padding: the remaining steps change nothing
    constexpr int b = S & 1, pq = P >> 2, pr = P & 3;
    gj_publish2<P>(v, rb, cb, colb, rowb);
    __syncthreads();
    // every LDS read of the step is issued first
    const double a = colb[b][0][P & 3][P >> 2], bb = colb[b][0][(P + 1) & 3][(P + 1) >> 2],
                 c = colb[b][1][(P + 1) & 3][(P + 1) >> 2];
    double c0[4], c1[4], R0[4], R1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        c0[i] = colb[b][0][i][rb];
        c1[i] = colb[b][1][i][rb];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        R0[j] = rowb[b][0][j][cb];
        R1[j] = rowb[b][1][j][cb];
    }
    __builtin_amdgcn_sched_barrier(0);
    const double det = __builtin_fma(a, c, -(bb * bb));
    if (!(a > 0.0 && det > 0.0)) ok = false;
    const double inv = recip(det);
    const double e00 = c * inv, e01 = -(bb * inv), e11 = a * inv;
    const bool prow = rb == pq, pcol = cb == pq;
    double W0[4], W1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        W0[i] = __builtin_fma(c0[i], -e00, c1[i] * -e01);   // -X(i, P) E
        W1[i] = __builtin_fma(c0[i], -e01, c1[i] * -e11);
    }
    W0[pr] = prow ? e00 : W0[pr];
    W1[pr] = prow ? e01 : W1[pr];
    W0[pr + 1] = prow ? e01 : W0[pr + 1];
    W1[pr + 1] = prow ? e11 : W1[pr + 1];
    R0[pr] = pcol ? 1.0 : R0[pr];
    R1[pr] = pcol ? 0.0 : R1[pr];
    R0[pr + 1] = pcol ? 0.0 : R0[pr + 1];
    R1[pr + 1] = pcol ? 1.0 : R1[pr + 1];
    const double mr = prow ? 0.0 : 1.0, mc = pcol ? 0.0 : 1.0, mrc = mr * mc;
    gj_entries2<pr>(std::make_integer_sequence<int, 16>{}, v, W0, W1, R0, R1, mr, mc, mrc);
}

template <int... S>
__device__ __forceinline__ void gj_steps2(std::integer_sequence<int, S...>, double (&v)[4][4], bool &ok, int w,
                                          int rb, int cb, double (*colb)[2][4][16], double (*rowb)[2][4][16]) {
    (gj_step2<S>(v, ok, w, rb, cb, colb, rowb), ...);
}

// LDS of the panel kernel; the pivot buffers first, so that their
// addresses fit the LDS instructions' immediate offsets
struct GjPanelLds {
    double colb[2][2][4][16];
    double rowb[2][2][4][16];
    double X[GJ_NB][GJ_LD];
    double Bl[GJ_NB][GJ_LD];
};

__device__ bool gj_invert_block(double (*X)[GJ_LD], int w, double (*colb)[2][4][16], double (*rowb)[2][4][16]) {
    const int tid = threadIdx.x;
    const int rb = tid & 15, cb = tid >> 4;
    __syncthreads();
    double v[4][4];   // v[i][j] = X(4 rb + i, 4 cb + j)
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i][j] = X[4 * cb + j][4 * rb + i];
    gj_steps2(std::make_integer_sequence<int, GJ_NB / 2>{}, v, ok, w, rb, cb, colb, rowb);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) X[4 * cb + j][4 * rb + i] = v[i][j];
    __syncthreads();
    return ok;   // uniform: every thread read the same pivots
}

__global__ __launch_bounds__(256) void gj_panel_kernel(const double *__restrict__ B, long ldb, Dim rd, int b,
                                                       double *__restrict__ Dbuf, double *__restrict__ Rrow,
                                                       double *__restrict__ Ccol, long ldc, int *status) {
    __shared__ __align__(16) GjPanelLds sh;
    double(*X)[GJ_LD] = sh.X;
    double(*Bl)[GJ_LD] = sh.Bl;
    const int r = rd.get();
    const int nbk = (r + GJ_NB - 1) / GJ_NB;
    const int jb = blockIdx.x;
    if (b >= nbk || jb >= nbk) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wb = min(GJ_NB, r - b * GJ_NB);
    const int wj = min(GJ_NB, r - jb * GJ_NB);
    const long ob = (long)b * GJ_NB, oj = (long)jb * GJ_NB;

    // all loads first (no branches), then the LDS and global writes.  Only
    // the lower block triangle of B is kept (diagonal blocks in full), so
    // block (jb, b) of the old block column is block (jb, b) itself for
    // jb >= b and the transpose of block (b, jb) for jb < b; either is read
    // coalesced, and Bl gets the pivot block row's block (b, jb) =
    // block (jb, b)'.
    const bool below = jb >= b;
    double xb[GJ_NB / 4], cb[GJ_NB / 4];
#pragma unroll
    for (int q = 0; q < GJ_NB / 4; ++q) {
        const int jc = wave + 4 * q;
        xb[q] = ld_or(B, (ob + lane) + (ob + jc) * ldb, lane < wb && jc < wb, lane == jc ? 1.0 : 0.0);
        // below: element (lane, jc) of block (jb, b); else of block (b, jb)
        cb[q] = below ? ld_or(B, (oj + lane) + (ob + jc) * ldb, lane < wj && jc < wb, 0.0)
                      : ld_or(B, (ob + lane) + (oj + jc) * ldb, lane < wb && jc < wj, 0.0);
    }
#pragma unroll
    for (int q = 0; q < GJ_NB / 4; ++q) {
        const int jc = wave + 4 * q;
        X[jc][lane] = xb[q];
        if (below) {
            if (lane < wj && jc < wb) Ccol[(oj + lane) + (long)jc * ldc] = cb[q];
            Bl[lane][jc] = jb != b ? cb[q] : 0.0;
        } else {
            Bl[jc][lane] = cb[q];
        }
    }
    const bool ok = gj_invert_block(X, wb, sh.colb, sh.rowb);   // begins and ends with a workgroup barrier
    if (!below) {
        // the old block column's block jb from the transpose in LDS
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            const int jc = wave + 4 * q;
            if (lane < wj && jc < wb) Ccol[(oj + lane) + (long)jc * ldc] = Bl[lane][jc];
        }
    }
    if (jb == b) {
        if (!ok && tid == 0) *status = ST_NOTSPD;
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            const int jc = wave + 4 * q;
            if (lane < wb && jc < wb) Dbuf[lane + (long)jc * GJ_NB] = X[jc][lane];
        }
        return;
    }
    // R = D * B_b,jb  (wb x wj)
    d4 acc[2][2];
    tile64_mfma(X, Bl, acc);
    const int wm = wave & 1, wn = wave >> 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * 32 + a * 16 + (lane & 15);
                const int col = wn * 32 + bb * 16 + (lane >> 4) + 4 * v;
                if (row < wb && col < wj) Rrow[row + (oj + col) * GJ_NB] = acc[a][bb][v];
            }
}

// tile (ib, jb) of the in-place update
__global__ __launch_bounds__(256) void gj_update_kernel(double *__restrict__ B, long ldb, Dim rd, int b,
                                                        const double *__restrict__ Dbuf,
                                                        const double *__restrict__ Rrow,
                                                        const double *__restrict__ Ccol, long ldc) {
    __shared__ double Xs[GJ_NB][GJ_LD];   // Xs[k][i]: left factor, column k
    __shared__ double Ys[GJ_NB][GJ_LD];   // Ys[j][k]: right factor, column j
    const int r = rd.get();
    const int nbk = (r + GJ_NB - 1) / GJ_NB;
    const int ib = blockIdx.x, jb = blockIdx.y;
    if (b >= nbk || ib >= nbk || jb >= nbk || ib < jb) return;   // the lower block triangle only
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wb = min(GJ_NB, r - b * GJ_NB);
    const int wi = min(GJ_NB, r - ib * GJ_NB);
    const int wj = min(GJ_NB, r - jb * GJ_NB);
    const long oi = (long)ib * GJ_NB, oj = (long)jb * GJ_NB;
    double *T = B + oi + oj * ldb;

    if (ib == b) {
        // row block b: -D on the diagonal tile, R_jb left of it (loads first)
        const bool diag = jb == b;
        const double *src = diag ? Dbuf : Rrow + oj * GJ_NB;
        const int wc = diag ? wb : wj;
        double t[GJ_NB / 4];
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            const int jc = wave + 4 * q;
            t[q] = ld_or(src, lane + (long)jc * GJ_NB, lane < wb && jc < wc, 0.0);
        }
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            const int jc = wave + 4 * q;
            if (lane < wb && jc < wc) T[lane + (long)jc * ldb] = diag ? -t[q] : t[q];
        }
        return;
    }
    const bool newcol = jb == b;
    const int wr = newcol ? wb : wj;
    // right factor: D (new block column) or R_jb
    const double *Y = newcol ? Dbuf : Rrow + oj * GJ_NB;
    const int wm = wave & 1, wn = wave >> 1;
    // every load first: both factors and the tile's old values (unless it is
    // overwritten), so that they are all in flight together
    double xv[GJ_NB / 4], yv[GJ_NB / 4], old[2][2][4];
#pragma unroll
    for (int q = 0; q < GJ_NB / 4; ++q) {
        const int kc = wave + 4 * q;
        // left factor: old block column rows of block ib (wi x wb), zero padded
        xv[q] = ld_or(Ccol, (oi + lane) + (long)kc * ldc, lane < wi && kc < wb, 0.0);
        yv[q] = ld_or(Y, lane + (long)kc * GJ_NB, lane < wb && kc < wr, 0.0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * 32 + a * 16 + (lane & 15);
                const int col = wn * 32 + bb * 16 + (lane >> 4) + 4 * v;
                old[a][bb][v] = ld_or(T, row + (long)col * ldb, !newcol && row < wi && col < wr, 0.0);
            }
#pragma unroll
    for (int q = 0; q < GJ_NB / 4; ++q) {
        const int kc = wave + 4 * q;
        Xs[kc][lane] = xv[q];
        Ys[kc][lane] = yv[q];
    }
    __syncthreads();
    d4 acc[2][2];
    tile64_mfma(Xs, Ys, acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * 32 + a * 16 + (lane & 15);
                const int col = wn * 32 + bb * 16 + (lane >> 4) + 4 * v;
                if (row < wi && col < wr)
                    T[row + (long)col * ldb] = newcol ? acc[a][bb][v] : old[a][bb][v] - acc[a][bb][v];
            }
}

hipError_t launch_gj_panel(const double *B, long ldb, Dim r, int b, double *D, double *Rrow, double *Ccol,
                           int *status, hipStream_t s) {
    const int nbk = (r.host + GJ_NB - 1) / GJ_NB;
    if (nbk <= 0) return hipSuccess;
    hipLaunchKernelGGL(gj_panel_kernel, dim3(nbk), dim3(256), 0, s, B, ldb, r, b, D, Rrow, Ccol,
                       (long)r.host, status);
    return hipGetLastError();
}

hipError_t launch_gj_update(double *B, long ldb, Dim r, int b, const double *D, const double *Rrow,
                            const double *Ccol, hipStream_t s) {
    const int nbk = (r.host + GJ_NB - 1) / GJ_NB;
    if (nbk <= 0) return hipSuccess;
    hipLaunchKernelGGL(gj_update_kernel, dim3(nbk, nbk), dim3(256), 0, s, B, ldb, r, b, D, Rrow, Ccol,
                       (long)r.host);
    return hipGetLastError();
}

// After the last sweep the lower triangle holds -B^-1: negate it and copy it
// to the upper triangle (32 x 32 tiles through LDS, one workgroup per tile on
// or below the diagonal).
__global__ void gj_finish_kernel(double *X, long ldx, Dim nd) {
    __shared__ double t[32][33];
    const int n = nd.get();
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bi < bj) return;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = bi * 32 + tx, j = bj * 32 + ty + 8 * q;
        v[q] = -ld_or(X, i + (long)j * ldx, i < n && j < n, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = bi * 32 + tx, j = bj * 32 + ty + 8 * q;
        if (i < n && j < n && i >= j) X[i + (long)j * ldx] = v[q];
        t[ty + 8 * q][tx] = v[q];
    }
    __syncthreads();
    for (int yy = ty; yy < 32; yy += 8) {
        const int di = bj * 32 + tx;   // destination row = source column
        const int dj = bi * 32 + yy;   // destination column = source row
        if (di < n && dj < n && dj > di) X[di + (long)dj * ldx] = t[tx][yy];
    }
}

hipError_t launch_gj_finish(double *X, long ldx, Dim n, hipStream_t s) {
    if (n.host <= 0) return hipSuccess;
    const int nt = (n.host + 31) / 32;
    hipLaunchKernelGGL(gj_finish_kernel, dim3(nt, nt), dim3(32, 8), 0, s, X, ldx, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Newton-Schulz iteration X <- X (2I - B X) for the inverse of an SPD matrix
// (the parallel-inverse alternative to the Gauss-Jordan sweep): the two
// products per step run on the float64 GEMM; these kernels set X_0 = a I,
// form 2I - T from T = B X while summing the squared residual (I - T), and
// the squared Frobenius norm of B.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ns_scaled_eye_kernel(double *X, long ldx, int n, double a) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i < n && j < n) X[i + (long)j * ldx] = i == j ? a : 0.0;
}

// sum2 += sum over the block of v^2 (one atomic per workgroup)
__device__ __forceinline__ void block_sum_sq(double v, double *sum2) {
    __shared__ double red[256];
    red[threadIdx.x] = v * v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(sum2, red[0]);
}

__global__ __launch_bounds__(256) void ns_two_minus_kernel(double *T, long ldt, int n, double *sum2) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    double d = 0.0;
    if (i < n && j < n) {
        const double t = T[i + (long)j * ldt];
        const double e = i == j ? 1.0 : 0.0;
        d = e - t;
        T[i + (long)j * ldt] = 2.0 * e - t;
    }
    block_sum_sq(d, sum2);
}

__global__ __launch_bounds__(256) void fro2_kernel(const double *B, long ldb, int n, double *sum2) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    block_sum_sq(i < n && j < n ? B[i + (long)j * ldb] : 0.0, sum2);
}

hipError_t launch_ns_scaled_eye(double *X, long ldx, int n, double a, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ns_scaled_eye_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, X, ldx, n, a);
    return hipGetLastError();
}

hipError_t launch_ns_two_minus(double *T, long ldt, int n, double *sum2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ns_two_minus_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, T, ldt, n, sum2);
    return hipGetLastError();
}

hipError_t launch_fro2(const double *B, long ldb, int n, double *sum2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fro2_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, B, ldb, n, sum2);
    return hipGetLastError();
}

}  // namespace geninv
