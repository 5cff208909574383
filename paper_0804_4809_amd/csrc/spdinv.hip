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
// whole elimination, so that a step needs only 4 entries of the pivot row
// and 4 of the pivot column per thread (broadcast LDS reads cost the full
// LDS return bandwidth, so the volume per step is what bounds it).  Those are
// published through LDS, double buffered by the parity of p (a buffer is
// rewritten two steps later, after every thread has passed the barrier of
// the step in between), so one barrier per step suffices.  Step p with
// d = 1 / X(p, p):
//   X(i, j) -= X(i, p) d X(p, j)   (i, j != p),   X(p, j) *= d   (j != p),
//   X(i, p) = -X(i, p) d           (i != p),      X(p, p) = d,
// written per element as v alpha + X(p, j) beta with (alpha, beta) = (1,
// -X(i, p) d) off row p and (d, 0) on it.  On return X holds the inverse.
// Returns false (uniformly) if a pivot is not positive.
//
// Only row and column p + 1 (mod 4) of every register block take step p's
// update at once: they hold what step p + 1 publishes.  The other nine
// entries take it after step p + 1's barrier, while that step's LDS reads
// are in flight, so the chain from one barrier to the next carries seven
// updates instead of sixteen.  Every entry still receives the same
// operations in the same order.
struct GjPending {
    double beta[4];   // -X(i, p) d for the thread's rows
    double rp[4];     // X(p, j) for the thread's columns
    double d;
};
struct GjRegs {
    double v[4][4];   // v[i][j] = X(4 rb + i, 4 cb + j)
    bool ok;
    GjPending pend[2];   // factors of step p, in slot p mod 2
};

// the update of entry (I, J) of the register block by a step whose pivot
// is row / column PR of the register blocks with rb / cb = pq (prow: rb ==
// pq, pcol: cb == pq)
template <int PR, int I, int J>
__device__ __forceinline__ void gj_entry(double &x, const GjPending &f, bool prow, bool pcol) {
    const bool onrow = I == PR && prow;
    const double alpha = onrow ? f.d : 1.0;
    const double be = onrow ? 0.0 : f.beta[I];
    x = __builtin_fma(f.rp[J], be, x * alpha);
    if (J == PR && pcol) x = onrow ? f.d : be;
}

// that update of the entries (I, J) with (I == R || J == R) == NEAR
template <int PR, int R, bool NEAR, int... E>
__device__ __forceinline__ void gj_entries(std::integer_sequence<int, E...>, double (&v)[4][4], const GjPending &f,
                                           bool prow, bool pcol) {
    ((((E >> 2) == R || (E & 3) == R) == NEAR ? gj_entry<PR, (E >> 2), (E & 3)>(v[E >> 2][E & 3], f, prow, pcol)
                                               : void()),
     ...);
}

// publish row and column p of the thread's register block (the threads that
// hold them) into buffer p mod 2
template <int P>
__device__ __forceinline__ void gj_publish(const GjRegs &g, int rb, int cb, double (*colb)[GJ_NB],
                                           double (*rowb)[GJ_NB]) {
    constexpr int b = P & 1, pq = P >> 2, pr = P & 3;
    if (cb == pq) {
#pragma unroll
        for (int i = 0; i < 4; ++i) colb[b][4 * rb + i] = g.v[i][pr];   // column p
    }
    if (rb == pq) {
#pragma unroll
        for (int j = 0; j < 4; ++j) rowb[b][4 * cb + j] = g.v[pr][j];   // row p
    }
}

constexpr auto gj_all = std::make_integer_sequence<int, 16>{};

// keeps x's computation before this point (the compiler would otherwise
// sink an update to its next use, past the following step's barrier)
__device__ __forceinline__ void gj_pin(double &x) { asm volatile("" : "+v"(x)); }

template <int R, int... E>
__device__ __forceinline__ void gj_pin_far(std::integer_sequence<int, E...>, double (&v)[4][4]) {
    (((E >> 2) != R && (E & 3) != R ? gj_pin(v[E >> 2][E & 3]) : void()), ...);
}

template <int P>
__device__ __forceinline__ void gj_step(GjRegs &g, int w, int rb, int cb, double (*colb)[GJ_NB],
                                        double (*rowb)[GJ_NB]) {
    if (P >= w) return;   // identity padding: the remaining steps change nothing
    constexpr int b = P & 1, pr = P & 3, nr = (P + 1) & 3;
    __syncthreads();
    // every LDS read of the step is issued first
    const double pv = colb[b][P];
    double cp[4];
    GjPending &f = g.pend[P & 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) cp[i] = colb[b][4 * rb + i];
#pragma unroll
    for (int j = 0; j < 4; ++j) f.rp[j] = rowb[b][4 * cb + j];
    __builtin_amdgcn_sched_barrier(0);
    // the previous step's pending update (entries off row and column p mod 4)
    if constexpr (P > 0) {
        constexpr int qq = (P - 1) >> 2;
        gj_entries<(P - 1) & 3, pr, false>(gj_all, g.v, g.pend[(P - 1) & 1], rb == qq, cb == qq);
        gj_pin_far<pr>(gj_all, g.v);
    }
    __builtin_amdgcn_sched_barrier(0);   // ... issued while the reads are in flight
    if (!(pv > 0.0)) g.ok = false;
    f.d = recip(pv);
#pragma unroll
    for (int i = 0; i < 4; ++i) f.beta[i] = -(cp[i] * f.d);
    // row and column p + 1 mod 4 now, then publish what step p + 1 reads
    gj_entries<pr, nr, true>(gj_all, g.v, f, rb == (P >> 2), cb == (P >> 2));
    gj_publish<P + 1>(g, rb, cb, colb, rowb);
}

template <int... P>
__device__ __forceinline__ void gj_steps(std::integer_sequence<int, P...>, GjRegs &g, int w, int rb, int cb,
                                         double (*colb)[GJ_NB], double (*rowb)[GJ_NB]) {
    (gj_step<P>(g, w, rb, cb, colb, rowb), ...);
}

// the pending update of the last step q (q mod 4 = QR)
template <int QR>
__device__ __forceinline__ void gj_flush(GjRegs &g, int q, int rb, int cb) {
    gj_entries<QR, (QR + 1) & 3, false>(gj_all, g.v, g.pend[QR & 1], rb == (q >> 2), cb == (q >> 2));
}

__device__ bool gj_invert_block(double (*X)[GJ_LD], int w) {
    __shared__ __align__(16) double colb[2][GJ_NB];
    __shared__ __align__(16) double rowb[2][GJ_NB];
    const int tid = threadIdx.x;
    const int rb = tid & 15, cb = tid >> 4;
    __syncthreads();
    GjRegs g;
    g.ok = true;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) g.v[i][j] = X[4 * cb + j][4 * rb + i];
    if (w > 0) {   // uniform
        gj_publish<0>(g, rb, cb, colb, rowb);
        gj_steps(std::make_integer_sequence<int, GJ_NB>{}, g, w, rb, cb, colb, rowb);
        const int q = w - 1;   // the last step
        switch (q & 3) {
        case 0: gj_flush<0>(g, q, rb, cb); break;
        case 1: gj_flush<1>(g, q, rb, cb); break;
        case 2: gj_flush<2>(g, q, rb, cb); break;
        default: gj_flush<3>(g, q, rb, cb); break;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) X[4 * cb + j][4 * rb + i] = g.v[i][j];
    __syncthreads();
    return g.ok;   // uniform: every thread read the same pivots
}

__global__ __launch_bounds__(256) void gj_panel_kernel(const double *__restrict__ B, long ldb, Dim rd, int b,
                                                       double *__restrict__ Dbuf, double *__restrict__ Rrow,
                                                       double *__restrict__ Ccol, long ldc, int *status) {
    __shared__ double X[GJ_NB][GJ_LD];
    __shared__ double Bl[GJ_NB][GJ_LD];
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
    const bool ok = gj_invert_block(X, wb);   // begins and ends with a workgroup barrier
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
