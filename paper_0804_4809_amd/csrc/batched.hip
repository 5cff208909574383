// Batched least squares W_b = G_b^+ F_b for thousands of small, unevenly sized
// problems in one persistent launch (Section 1's least-squares use of the
// method, Section 4's many small fits; the method itself is the Appendix's).
// This launch takes the tall problems (m_b >= n_b); wide ones run in a second
// persistent launch with the Appendix's transpose branch (end of the file).
//
// Every workgroup (256 threads) takes problems from a device work queue (an
// atomic counter over a host-computed order, largest first) until the queue
// is empty; all workgroups reach that exit.  One problem runs entirely inside
// one workgroup:
//
//   1. A = G'G and B = G'F, float32 inputs accumulated in float64 (register
//      tiles of 8 x 4 outputs per thread, G staged through LDS 16 rows at a
//      time)
//   2. tol = 1e-9 min{A_kk > 0} (or the caller's), then the full-rank Cholesky
//      of A in place, column by column with the paper's strict test
//   3. C = L'L and T = L'B, as a second Gram product over the kept columns
//   4. M = C^-1 in place by Gauss-Jordan elimination (C is SPD)
//   5. W = L (M (M T))
//
// A (and later C) lives in LDS when its order is at most `nl` (a launch
// parameter chosen by the autotuner), otherwise in a per-workgroup slab of
// global memory; the same code runs on either through flat pointers.
#include "common.h"

namespace geninv {

constexpr int BT_THREADS = 256;
constexpr int BT_STAGE_ROWS = 16;

// LDS layouts against bank conflicts (the LDS serves 8-byte reads 16 lanes
// at a time over 32 four-byte banks).  A stage row keeps element c at
// c + c / 16 and has an odd pitch: the Gram's reads of four consecutive
// elements per thread (thread t at 4 t) then meet 16 distinct bank pairs, and
// the staging writes (16 rows at one element) too.  The blocked routines'
// panels (NB columns of consecutive rows) have an odd row pitch NB + 1.
__device__ __forceinline__ int stage_pos(int c) { return c + (c >> 4); }
__host__ __device__ constexpr int stage_pitch(int w) { return (w + ((w + 15) >> 4)) | 1; }

__device__ __forceinline__ double ldv(const float *p) { return (double)*p; }
__device__ __forceinline__ double ldv(const double *p) { return *p; }

// Lower triangle of X(:, cols)' X(:, cols) into Aout (nc x nc, lda) and
// X(:, cols)' F into Bout (nc x k, ldb).  cols[c] selects the source column of
// output column c (identity when cols == nullptr); with `tri`, the source is
// taken as zero above row cols[c] (a lower trapezoidal factor).
template <typename T>
__device__ __forceinline__ void block_gram(const T *X, long ldx, int rows, int nc, const int *cols, bool tri, const T *F, long ldf,
                           int k, double *Aout, long lda, double *Bout, long ldb, double *stage) {
    // a thread owns 8 output rows x 4 output columns: tiles (ti, tj) with
    // 4 tj <= 8 ti + 7 cover the lower triangle of X'X (2 ti + 2 of them in
    // row block ti), then the blocks of X'F
    const int tid = threadIdx.x;
    const int nt = (nc + 7) / 8, kt = (k + 3) / 4;
    const int tri_tiles = nt * (nt + 1);
    const int ntiles = tri_tiles + nt * kt;
    const int sw = nc + k;                 // stage width (columns)
    const int swp = stage_pitch(sw);
    for (int base = 0; base < ntiles; base += BT_THREADS) {
        const int t = base + tid;
        int ti = 0, tj = 0;
        bool fcol = false, active = t < ntiles;
        if (active) {
            if (t < tri_tiles) {
                ti = (int)((sqrtf(4.0f * t + 1.0f) - 1.0f) * 0.5f);
                while (ti * (ti + 1) > t) --ti;
                while ((ti + 1) * (ti + 2) <= t) ++ti;
                tj = t - ti * (ti + 1);
            } else {
                const int u = t - tri_tiles;
                ti = u / kt;
                tj = u % kt;
                fcol = true;
            }
        }
        double acc[8][4];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        // stage positions: 8 ti + a and 4 tj + b share their padding for
        // a < 8, b < 4 (F columns start at nc, anywhere: one per column)
        const int apos = 8 * ti + (ti >> 1);
        int bpos[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) bpos[b] = fcol ? stage_pos(nc + tj * 4 + b) : 4 * tj + (tj >> 2) + b;
        for (int k0 = 0; k0 < rows; k0 += BT_STAGE_ROWS) {
            __syncthreads();
            // branch-free loads (clamped address, then select) so that a
            // thread's loads of the stage issue back to back
            for (int e = tid; e < BT_STAGE_ROWS * sw; e += BT_THREADS) {
                const int r = e % BT_STAGE_ROWS, c = e / BT_STAGE_ROWS;
                const int row = k0 + r;
                const bool inx = c < nc;
                const int src = inx ? (cols ? cols[c] : c) : 0;
                const bool ok = row < rows && (!inx || !tri || row >= src);
                const T *p = inx ? X + row + (long)src * ldx : F + row + (long)(c - nc) * ldf;
                const double v = ldv(ok ? p : X);
                stage[r * swp + stage_pos(c)] = ok ? v : 0.0;
            }
            __syncthreads();
            if (active) {
#pragma unroll 4
                for (int r = 0; r < BT_STAGE_ROWS; ++r) {
                    double av[8], bv[4];
                    const double *srow = stage + r * swp;
#pragma unroll
                    for (int a = 0; a < 8; ++a) {
                        const int ci = ti * 8 + a;
                        av[a] = ci < nc ? srow[apos + a] : 0.0;
                    }
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int cj = fcol ? nc + tj * 4 + b : tj * 4 + b;
                        bv[b] = (fcol ? (tj * 4 + b < k) : (cj < nc)) ? srow[bpos[b]] : 0.0;
                    }
#pragma unroll
                    for (int a = 0; a < 8; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
                }
            }
        }
        if (active) {
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int i = ti * 8 + a, j = tj * 4 + b;
                    if (i >= nc) continue;
                    if (fcol) {
                        if (j < k) Bout[i + (long)j * ldb] = acc[a][b];
                    } else if (j <= i) {
                        Aout[i + (long)j * lda] = acc[a][b];
                    }
                }
        }
    }
    __syncthreads();
}

// tol (<= 0: paper default), returns the threshold; also flags non-finite diagonals
__device__ __forceinline__ double block_tol(const double *A, long lda, int n, double user_tol, double *red, int *bad) {
    const int tid = threadIdx.x;
    double mn = __builtin_huge_val();
    int b = 0;
    for (int i = tid; i < n; i += BT_THREADS) {
        const double a = A[i + (long)i * lda];
        if (!__builtin_isfinite(a)) b = 1;
        else if (a > 0.0 && a < mn) mn = a;
    }
    red[tid] = mn;
    __syncthreads();
    if (b) *bad = 1;
    for (int s = BT_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmin(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double m = red[0];
    __syncthreads();
    if (*bad) return __builtin_huge_val();
    if (user_tol > 0.0) return user_tol;
    return m == __builtin_huge_val() ? m : m * 1e-9;
}

// full-rank Cholesky in place on the lower triangle of A (n x n): column j
// kept iff its updated pivot is > tol.  Kept columns hold L (rows >= j), the
// others are zeroed.  cols[] receives the kept column indices; returns r.
__device__ __forceinline__ int block_frchol(double *A, long lda, int n, double tol, int *cols, int *cnt) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) *cnt = 0;
    for (int j = 0; j < n; ++j) {
        __syncthreads();
        const double d = A[j + (long)j * lda];
        const bool keep = d > tol;
        double *colj = A + (long)j * lda;
        __syncthreads();   // every thread has read the pivot before it is overwritten
        if (keep) {
            const double s = sqrt(d);
            for (int i = j + 1 + tid; i < n; i += BT_THREADS) colj[i] = colj[i] / s;
            if (tid == 0) {
                colj[j] = s;
                cols[*cnt] = j;
                *cnt = *cnt + 1;
            }
            __syncthreads();
            for (int l = j + 1 + wave; l < n; l += 4) {
                const double f = colj[l];
                double *coll = A + (long)l * lda;
                for (int i = l + lane; i < n; i += 64) coll[i] -= colj[i] * f;
            }
        } else {
            for (int i = j + tid; i < n; i += BT_THREADS) colj[i] = 0.0;
        }
    }
    __syncthreads();
    const int r = *cnt;
    __syncthreads();
    return r;
}

// The same full-rank Cholesky for A in global memory (the per-workgroup
// slab), in panels of NB columns: a panel (rows j0..n-1) is factored column
// by column in LDS (ws, n x NB, row pitch NB + 1) with the paper's strict test, written back,
// and the columns to its right take one rank-NB update (4 x 4 register
// tiles) instead of one update per column.  Decisions and kept values are
// those of the column-by-column form up to the grouping of the updates.
template <int NB>
__device__ __forceinline__ int block_frchol_blocked(double *A, long lda, int n, double tol, int *cols, int *cnt, double *ws) {
    const int tid = threadIdx.x;
    constexpr int PP = NB + 1;   // panel row pitch
    double *Ps = ws;   // Ps[i * PP + c] = A(i, j0 + c)
    if (tid == 0) *cnt = 0;
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int nb = min(NB, n - j0);
        __syncthreads();
        for (int e = tid; e < (n - j0) * nb; e += BT_THREADS) {
            const int i = j0 + e % (n - j0), c = e / (n - j0);
            Ps[i * PP + c] = i >= j0 + c ? A[i + (long)(j0 + c) * lda] : 0.0;
        }
        for (int c = 0; c < nb; ++c) {
            const int j = j0 + c;
            __syncthreads();
            const double d = Ps[j * PP + c];
            const bool keep = d > tol;
            __syncthreads();   // every thread has read the pivot before it is overwritten
            if (keep) {
                const double sq = sqrt(d);
                for (int i = j + 1 + tid; i < n; i += BT_THREADS) Ps[i * PP + c] /= sq;
                if (tid == 0) {
                    Ps[j * PP + c] = sq;
                    cols[*cnt] = j;
                    *cnt = *cnt + 1;
                }
                __syncthreads();
                // the panel's later columns: Ps(i, c2) -= L(i, j) L(j0 + c2, j), i >= j0 + c2
                for (int e = tid; e < (n - j0) * nb; e += BT_THREADS) {
                    const int i = j0 + e % (n - j0), c2 = e / (n - j0);
                    if (c2 > c && i >= j0 + c2) Ps[i * PP + c2] -= Ps[i * PP + c] * Ps[(j0 + c2) * PP + c];
                }
            } else {
                for (int i = j + tid; i < n; i += BT_THREADS) Ps[i * PP + c] = 0.0;
            }
        }
        __syncthreads();
        for (int e = tid; e < (n - j0) * nb; e += BT_THREADS) {
            const int i = j0 + e % (n - j0), c = e / (n - j0);
            if (i >= j0 + c) A[i + (long)(j0 + c) * lda] = Ps[i * PP + c];
        }
        // columns l >= j0 + nb, rows i >= l: A(i, l) -= sum_c L(i, j0 + c) L(l, j0 + c)
        const int t0 = j0 + nb, nt = (n - t0 + 3) / 4;
        for (int t = tid; t < nt * nt; t += BT_THREADS) {
            const int ti = t % nt, tl = t / nt;
            if (ti < tl) continue;   // tiles on or below the diagonal
            const int i0 = t0 + 4 * ti, l0 = t0 + 4 * tl;
            double q[4][NB];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < NB; ++c) q[a][c] = (c < nb && i0 + a < n) ? Ps[(i0 + a) * PP + c] : 0.0;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const int l = l0 + bb;
                if (l >= n) continue;
                double x[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) x[c] = c < nb ? Ps[l * PP + c] : 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int i = i0 + a;
                    if (i >= n || i < l) continue;
                    double sum = 0.0;
#pragma unroll
                    for (int c = 0; c < NB; ++c) sum = fma(q[a][c], x[c], sum);
                    A[i + (long)l * lda] -= sum;
                }
            }
        }
    }
    __syncthreads();
    const int r = *cnt;
    __syncthreads();
    return r;
}

// in-place Gauss-Jordan inverse of the SPD matrix C (r x r, full storage);
// returns false if a pivot is not positive
__device__ __forceinline__ bool block_gj(double *C, long ldc, int r, double *rowp, double *colp) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    bool ok = true;
    for (int p = 0; p < r; ++p) {
        __syncthreads();
        const double pv = C[p + (long)p * ldc];
        if (!(pv > 0.0)) ok = false;
        const double dinv = 1.0 / pv;
        for (int t = tid; t < r; t += BT_THREADS) {
            rowp[t] = C[p + (long)t * ldc] * dinv;
            colp[t] = C[t + (long)p * ldc];
        }
        __syncthreads();
        for (int jc = wave; jc < r; jc += 4) {
            const double rp = rowp[jc];
            double *colc = C + (long)jc * ldc;
            for (int i = lane; i < r; i += 64) {
                double v = colc[i] - colp[i] * rp;
                if (i == p) v = rp;
                if (jc == p) v = (i == p) ? dinv : -colp[i] * dinv;
                colc[i] = v;
            }
        }
    }
    __syncthreads();
    return ok;
}

// Blocked Gauss-Jordan for C in global memory (the per-workgroup slab): the
// same elimination as block_gj with pivot blocks of nb columns, so that C is
// read and rewritten once per block instead of once per pivot.  Per block
// (D = C_bb, Q = old block column, R = block row):
//   D^-1 in LDS;  R' = D^-1 R;  C_ij -= Q_i R'_j  (i, j outside the block);
//   C_bj = R'_j;  C_ib = -Q_i D^-1;  C_bb = D^-1.
// ws (LDS) holds Q (r x NB, row pitch NB + 1), R' (NB x r) and D (NB x NB).
// The pivot test's result is that of the first wavefront (the caller reads
// it on thread 0).
template <int NB>
__device__ __forceinline__ bool block_gj_blocked(double *C, long ldc, int r, double *ws) {
    const int tid = threadIdx.x;
    constexpr int QP = NB + 1;          // Qs row pitch
    double *Qs = ws;                    // Qs[i * QP + c] = C(i, b0 + c)
    double *Rs = Qs + (long)r * QP;     // Rs[c * r + j] = C(b0 + c, j), then R'
    double *Ds = Rs + (long)NB * r;     // Ds[c * NB + c'] = D(c, c'), then D^-1
    bool ok = true;
    for (int b0 = 0; b0 < r; b0 += NB) {
        const int nb = min(NB, r - b0);
        __syncthreads();
        for (int e = tid; e < r * nb; e += BT_THREADS) {
            const int i = e % r, c = e / r;
            Qs[i * QP + c] = C[i + (long)(b0 + c) * ldc];
        }
        for (int e = tid; e < nb * r; e += BT_THREADS) {
            const int c = e % nb, j = e / nb;
            Rs[c * r + j] = C[(b0 + c) + (long)j * ldc];
        }
        __syncthreads();
        for (int e = tid; e < nb * nb; e += BT_THREADS) {
            const int c = e % nb, c2 = e / nb;
            Ds[c * NB + c2] = Qs[(b0 + c) * QP + c2];
        }
        // D^-1 in place on the first wavefront, one pivot at a time: lane
        // c + NB c2 holds D(c, c2) (NB^2 <= 64), and a step's pivot row and
        // column come from the other lanes by shuffles, so the pivots need no
        // workgroup barrier
        __syncthreads();
        if (tid < 64) {
            const int c = tid % NB, c2 = tid / NB;
            const bool in = tid < NB * NB && c < nb && c2 < nb;
            double v = in ? Ds[c * NB + c2] : 0.0;
            for (int p = 0; p < nb; ++p) {
                const double pv = __shfl(v, p + NB * p, 64);
                const double drow = __shfl(v, p + NB * (c2 & (NB - 1)), 64);   // D(p, c2)
                const double dcol = __shfl(v, c + NB * p, 64);                  // D(c, p)
                if (!(pv > 0.0)) ok = false;
                const double dinv = 1.0 / pv;
                const double rp = drow * dinv, cp = dcol;
                v = (c == p) ? ((c2 == p) ? dinv : rp) : ((c2 == p) ? -cp * dinv : v - cp * rp);
            }
            if (in) Ds[c * NB + c2] = v;
        }
        __syncthreads();
        // R' = D^-1 R (registers first: R is read by every output)
        constexpr int NRR = NB * 256 / BT_THREADS;   // elements per thread for r <= 256
        double rn[NRR];
#pragma unroll
        for (int h = 0; h < NRR; ++h) {
            const int e = tid + h * BT_THREADS;
            rn[h] = 0.0;
            if (e < nb * r) {
                const int c = e % nb, j = e / nb;
                double acc = 0.0;
                for (int c2 = 0; c2 < nb; ++c2) acc = fma(Ds[c * NB + c2], Rs[c2 * r + j], acc);
                rn[h] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < NRR; ++h) {
            const int e = tid + h * BT_THREADS;
            if (e < nb * r) Rs[(e % nb) * r + e / nb] = rn[h];
        }
        __syncthreads();
        // every element of C, 4 x 4 per thread
        const int tr = (r + 3) / 4;
        for (int t = tid; t < tr * tr; t += BT_THREADS) {
            const int i0 = 4 * (t % tr), j0 = 4 * (t / tr);
            double q[4][NB];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < NB; ++c) q[a][c] = (c < nb && i0 + a < r) ? Qs[(i0 + a) * QP + c] : 0.0;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const int j = j0 + bb;
                if (j >= r) continue;
                const bool jin = j >= b0 && j < b0 + nb;
                double x[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) x[c] = c < nb ? (jin ? Ds[c * NB + (j - b0)] : Rs[c * r + j]) : 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int i = i0 + a;
                    if (i >= r) continue;
                    const bool iin = i >= b0 && i < b0 + nb;
                    double sum = 0.0;
#pragma unroll
                    for (int c = 0; c < NB; ++c) sum = fma(q[a][c], x[c], sum);
                    double xi = 0.0;   // x[i - b0] without a dynamically indexed register array
#pragma unroll
                    for (int c = 0; c < NB; ++c) xi = (c == i - b0) ? x[c] : xi;
                    double *cij = C + i + (long)j * ldc;
                    *cij = iin ? xi : (jin ? -sum : *cij - sum);
                }
            }
        }
    }
    __syncthreads();
    return ok;
}

struct BatchDesc {
    const float *G; const float *F; double *W;
    int *piv;            // optional: kept column indices (r of them), or null
    int m, n, ldg, ldf, ldw;
    int pad;
};

__global__ __launch_bounds__(BT_THREADS, 2) void batched_lstsq_kernel(const BatchDesc *desc, const int *order, int batch,
                                                                   int k, double user_tol, int nl, int *queue,
                                                                   double *slabs, long slab_stride, int nmax,
                                                                   int *rank, int *status) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    // LDS carve-up: [nl*nl] big | [16*stage_pitch(nmax+k)] stage | [256] red | [nmax] rowp | [nmax] colp | ints
    double *big = lds;
    double *stage = big + (long)nl * nl;
    double *red = stage + BT_STAGE_ROWS * stage_pitch(nmax + k);
    double *rowp = red + BT_THREADS;
    double *colp = rowp + nmax;
    int *cols = reinterpret_cast<int *>(colp + nmax);
    int *ints = cols + nmax;            // [0] queue slot, [1] counter, [2] bad flag

    double *slab = slabs + (long)blockIdx.x * slab_stride;
    double *Lg = slab;                                   // nmax x nmax
    double *Cg = Lg + (long)nmax * nmax;                 // nmax x nmax
    double *Bv = Cg + (long)nmax * nmax;                 // nmax x k: G'F
    double *Tv = Bv + (long)nmax * k;                    // nmax x k: L'B, then M x
    double *Xv = Tv + (long)nmax * k;                    // nmax x k

    const int tid = threadIdx.x;
    // The blocked Cholesky and Gauss-Jordan keep their panels in the LDS
    // matrix region and the staging rows behind it (contiguous, and both
    // idle while A or L'L lives in the slab).  Block width 8 or 4, whichever
    // is the larger that fits: panels of nmax (NB + 1) doubles (Cholesky),
    // nmax (2 NB + 1) + NB^2 (Gauss-Jordan).
    const long ws_cap = (long)nl * nl + (long)BT_STAGE_ROWS * stage_pitch(nmax + k);
    int gj_nb = 0, fr_nb = 0;
    for (int nbc = 8; nbc >= 4; nbc /= 2) {
        if (gj_nb == 0 && ws_cap >= (long)nmax * (2 * nbc + 1) + (long)nbc * nbc) gj_nb = nbc;
        if (fr_nb == 0 && ws_cap >= (long)nmax * (nbc + 1)) fr_nb = nbc;
    }
    for (;;) {
        if (tid == 0) ints[0] = atomicAdd(queue, 1);
        __syncthreads();
        const int slot = ints[0];
        __syncthreads();
        if (slot >= batch) break;
        const int b = order[slot];
        const BatchDesc d = desc[b];
        const int m = d.m, n = d.n;
        if (tid == 0) ints[2] = 0;

        // 1. A = G'G, B = G'F
        double *A = (n <= nl) ? big : Lg;
        const long lda = n;
        block_gram<float>(d.G, d.ldg, m, n, nullptr, false, d.F, d.ldf, k, A, lda, Bv, n, stage);
        // 2. tolerance and full-rank Cholesky in place
        const double tol = block_tol(A, lda, n, user_tol, red, &ints[2]);
        if (ints[2] && tid == 0) *status = ST_NONFINITE;
        const int r = (A == Lg && fr_nb == 8)   ? block_frchol_blocked<8>(A, lda, n, tol, cols, &ints[1], big)
                      : (A == Lg && fr_nb == 4) ? block_frchol_blocked<4>(A, lda, n, tol, cols, &ints[1], big)
                                                : block_frchol(A, lda, n, tol, cols, &ints[1]);
        if (tid == 0) rank[b] = r;
        if (d.piv)
            for (int c = tid; c < r; c += BT_THREADS) d.piv[c] = cols[c];
        if (r == 0) {
            for (int e = tid; e < n * k; e += BT_THREADS) d.W[(e % n) + (long)(e / n) * d.ldw] = 0.0;
            __syncthreads();
            continue;
        }
        // L must stay readable while C occupies LDS: move it to the slab
        if (A == big) {
            for (long e = tid; e < (long)n * n; e += BT_THREADS) Lg[e] = big[e];
            __syncthreads();
        }
        // 3. C = L'L (kept columns), T = L'B
        double *C = (r <= nl) ? big : Cg;
        const long ldc = r;
        block_gram<double>(Lg, n, n, r, cols, true, Bv, n, k, C, ldc, Tv, r, stage);
        // full symmetric C from its lower triangle
        for (long e = tid; e < (long)r * r; e += BT_THREADS) {
            const int i = (int)(e % r), j = (int)(e / r);
            if (i < j) C[i + (long)j * ldc] = C[j + (long)i * ldc];
        }
        __syncthreads();
        // 4. M = C^-1: blocked when C is in the slab (panels in the LDS matrix
        // region and staging rows)
        const bool ok = (C == Cg && gj_nb == 8)   ? block_gj_blocked<8>(C, ldc, r, big)
                        : (C == Cg && gj_nb == 4) ? block_gj_blocked<4>(C, ldc, r, big)
                                                  : block_gj(C, ldc, r, rowp, colp);
        if (!ok && tid == 0) *status = ST_NOTSPD;
        // 5. X = M T, T = M X, W = L T
        for (int e = tid; e < r * k; e += BT_THREADS) {
            const int i = e % r, q = e / r;
            double s = 0.0;
            for (int j = 0; j < r; ++j) s = fma(C[i + (long)j * ldc], Tv[j + (long)q * r], s);
            Xv[i + (long)q * r] = s;
        }
        __syncthreads();
        for (int e = tid; e < r * k; e += BT_THREADS) {
            const int i = e % r, q = e / r;
            double s = 0.0;
            for (int j = 0; j < r; ++j) s = fma(C[i + (long)j * ldc], Xv[j + (long)q * r], s);
            Tv[i + (long)q * r] = s;
        }
        __syncthreads();
        for (int e = tid; e < n * k; e += BT_THREADS) {
            const int i = e % n, q = e / n;
            double s = 0.0;
            for (int c = 0; c < r && cols[c] <= i; ++c) s = fma(Lg[i + (long)cols[c] * n], Tv[c + (long)q * r], s);
            d.W[i + (long)q * d.ldw] = s;
        }
        __syncthreads();
    }
}

__global__ void reset_queue_kernel(int *q) {
    if (threadIdx.x == 0) *q = 0;
}

size_t batched_lds_bytes(int nl, int nmax, int k) {
    return sizeof(double) * ((size_t)nl * nl + (size_t)BT_STAGE_ROWS * stage_pitch(nmax + k) + BT_THREADS +
                             2 * (size_t)nmax) +
           sizeof(int) * ((size_t)nmax + 4);
}

size_t batched_slab_doubles(int nmax, int k) {
    return 2 * (size_t)nmax * nmax + 3 * (size_t)nmax * k;
}

hipError_t launch_batched(const void *desc, const int *order, int batch, int k, double tol, int nl, int *queue,
                          double *slabs, int grid, int nmax, int *rank, int *status, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = batched_lds_bytes(nl, nmax, k);
    hipLaunchKernelGGL(batched_lstsq_kernel, dim3(grid), dim3(BT_THREADS), lds, s,
                       static_cast<const BatchDesc *>(desc), order, batch, k, tol, nl, queue, slabs,
                       (long)batched_slab_doubles(nmax, k), nmax, rank, status);
    return hipGetLastError();
}

size_t batched_desc_bytes() { return sizeof(BatchDesc); }

void batched_fill_desc(void *out, const float *G, const float *F, double *W, int m, int n, int ldg, int ldf, int ldw) {
    BatchDesc *d = static_cast<BatchDesc *>(out);
    d->G = G; d->F = F; d->W = W;
    d->piv = nullptr;
    d->m = m; d->n = n; d->ldg = ldg; d->ldf = ldf; d->ldw = ldw;
    d->pad = 0;
}

void batched_set_piv(void *desc, int b, int *piv) { static_cast<BatchDesc *>(desc)[b].piv = piv; }

// ---------------------------------------------------------------------------
// Wide problems (m_b < n_b): the Appendix's transpose branch, one problem per
// workgroup as above.  The m x m matrix G G' is factored (its lower triangle
// from the rows of G, staged 16 columns of G at a time), B = F, and after
// X = M (M (L' F)) the weights are W = G' (L X).  A separate kernel, so that
// the tall problems' kernel stays as it is.
// ---------------------------------------------------------------------------

// Lower triangle of G G' (m x m, lda) for G m x n (ldg): the stage holds
// columns k0 .. k0 + 15 of G as rows, 8 x 4 output tiles per thread.
__device__ __forceinline__ void block_gram_rows(const float *G, long ldg, int m, int n, double *Aout, long lda, double *stage) {
    const int tid = threadIdx.x;
    const int nt = (m + 7) / 8;
    const int ntiles = nt * (nt + 1);
    const int swp = stage_pitch(m);
    for (int base = 0; base < ntiles; base += BT_THREADS) {
        const int t = base + tid;
        int ti = 0, tj = 0;
        const bool active = t < ntiles;
        if (active) {
            ti = (int)((sqrtf(4.0f * t + 1.0f) - 1.0f) * 0.5f);
            while (ti * (ti + 1) > t) --ti;
            while ((ti + 1) * (ti + 2) <= t) ++ti;
            tj = t - ti * (ti + 1);
        }
        double acc[8][4];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        const int apos = 8 * ti + (ti >> 1), bpos = 4 * tj + (tj >> 2);   // stage positions of 8 ti and 4 tj
        for (int k0 = 0; k0 < n; k0 += BT_STAGE_ROWS) {
            __syncthreads();
            // stage row r = column k0 + r of G (m consecutive floats)
            for (int e = tid; e < BT_STAGE_ROWS * m; e += BT_THREADS) {
                const int c = e % m, r = e / m;
                const bool ok = k0 + r < n;
                const double v = (double)G[ok ? c + (long)(k0 + r) * ldg : 0];
                stage[r * swp + stage_pos(c)] = ok ? v : 0.0;
            }
            __syncthreads();
            if (active) {
#pragma unroll 4
                for (int r = 0; r < BT_STAGE_ROWS; ++r) {
                    double av[8], bv[4];
                    const double *srow = stage + r * swp;
#pragma unroll
                    for (int a = 0; a < 8; ++a) {
                        const int ci = ti * 8 + a;
                        av[a] = ci < m ? srow[apos + a] : 0.0;
                    }
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int cj = tj * 4 + b;
                        bv[b] = cj < m ? srow[bpos + b] : 0.0;
                    }
#pragma unroll
                    for (int a = 0; a < 8; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
                }
            }
        }
        if (active) {
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int i = ti * 8 + a, j = tj * 4 + b;
                    if (i < m && j <= i) Aout[i + (long)j * lda] = acc[a][b];
                }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(BT_THREADS, 2) void batched_wide_kernel(const BatchDesc *desc, const int *order, int batch,
                                                                  int k, double user_tol, int nl, int *queue,
                                                                  double *slabs, long slab_stride, int nmax,
                                                                  int *rank, int *status) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    double *big = lds;
    double *stage = big + (long)nl * nl;
    double *red = stage + BT_STAGE_ROWS * stage_pitch(nmax + k);
    double *rowp = red + BT_THREADS;
    double *colp = rowp + nmax;
    int *cols = reinterpret_cast<int *>(colp + nmax);
    int *ints = cols + nmax;

    double *slab = slabs + (long)blockIdx.x * slab_stride;
    double *Lg = slab;
    double *Cg = Lg + (long)nmax * nmax;
    double *Bv = Cg + (long)nmax * nmax;
    double *Tv = Bv + (long)nmax * k;
    double *Xv = Tv + (long)nmax * k;

    const int tid = threadIdx.x;
    const long ws_cap = (long)nl * nl + (long)BT_STAGE_ROWS * stage_pitch(nmax + k);
    int gj_nb = 0, fr_nb = 0;
    for (int nbc = 8; nbc >= 4; nbc /= 2) {
        if (gj_nb == 0 && ws_cap >= (long)nmax * (2 * nbc + 1) + (long)nbc * nbc) gj_nb = nbc;
        if (fr_nb == 0 && ws_cap >= (long)nmax * (nbc + 1)) fr_nb = nbc;
    }
    for (;;) {
        if (tid == 0) ints[0] = atomicAdd(queue, 1);
        __syncthreads();
        const int slot = ints[0];
        __syncthreads();
        if (slot >= batch) break;
        const int b = order[slot];
        const BatchDesc d = desc[b];
        const int m = d.m, n = d.n;   // m < n: the factored order is m
        if (tid == 0) ints[2] = 0;

        // 1. A = G G' (m x m), B = F
        double *A = (m <= nl) ? big : Lg;
        const long lda = m;
        block_gram_rows(d.G, d.ldg, m, n, A, lda, stage);
        for (int e = tid; e < m * k; e += BT_THREADS) Bv[e] = (double)d.F[(e % m) + (long)(e / m) * d.ldf];
        __syncthreads();
        // 2. tolerance and full-rank Cholesky in place
        const double tol = block_tol(A, lda, m, user_tol, red, &ints[2]);
        if (ints[2] && tid == 0) *status = ST_NONFINITE;
        const int r = (A == Lg && fr_nb == 8)   ? block_frchol_blocked<8>(A, lda, m, tol, cols, &ints[1], big)
                      : (A == Lg && fr_nb == 4) ? block_frchol_blocked<4>(A, lda, m, tol, cols, &ints[1], big)
                                                : block_frchol(A, lda, m, tol, cols, &ints[1]);
        if (tid == 0) rank[b] = r;
        if (d.piv)
            for (int c = tid; c < r; c += BT_THREADS) d.piv[c] = cols[c];
        if (r == 0) {
            for (int e = tid; e < n * k; e += BT_THREADS) d.W[(e % n) + (long)(e / n) * d.ldw] = 0.0;
            __syncthreads();
            continue;
        }
        if (A == big) {
            for (long e = tid; e < (long)m * m; e += BT_THREADS) Lg[e] = big[e];
            __syncthreads();
        }
        // 3. C = L'L (kept columns), T = L'F
        double *C = (r <= nl) ? big : Cg;
        const long ldc = r;
        block_gram<double>(Lg, m, m, r, cols, true, Bv, m, k, C, ldc, Tv, r, stage);
        for (long e = tid; e < (long)r * r; e += BT_THREADS) {
            const int i = (int)(e % r), j = (int)(e / r);
            if (i < j) C[i + (long)j * ldc] = C[j + (long)i * ldc];
        }
        __syncthreads();
        // 4. M = C^-1
        const bool ok = (C == Cg && gj_nb == 8)   ? block_gj_blocked<8>(C, ldc, r, big)
                        : (C == Cg && gj_nb == 4) ? block_gj_blocked<4>(C, ldc, r, big)
                                                  : block_gj(C, ldc, r, rowp, colp);
        if (!ok && tid == 0) *status = ST_NOTSPD;
        // 5. X = M T, T = M X, V = L T (m x k, into Xv), W = G' V
        for (int e = tid; e < r * k; e += BT_THREADS) {
            const int i = e % r, q = e / r;
            double s = 0.0;
            for (int j = 0; j < r; ++j) s = fma(C[i + (long)j * ldc], Tv[j + (long)q * r], s);
            Xv[i + (long)q * r] = s;
        }
        __syncthreads();
        for (int e = tid; e < r * k; e += BT_THREADS) {
            const int i = e % r, q = e / r;
            double s = 0.0;
            for (int j = 0; j < r; ++j) s = fma(C[i + (long)j * ldc], Xv[j + (long)q * r], s);
            Tv[i + (long)q * r] = s;
        }
        __syncthreads();
        for (int e = tid; e < m * k; e += BT_THREADS) {
            const int i = e % m, q = e / m;
            double s = 0.0;
            for (int c = 0; c < r && cols[c] <= i; ++c) s = fma(Lg[i + (long)cols[c] * m], Tv[c + (long)q * r], s);
            Xv[i + (long)q * m] = s;
        }
        __syncthreads();
        for (int e = tid; e < n * k; e += BT_THREADS) {
            const int j = e % n, q = e / n;
            const float *gj = d.G + (long)j * d.ldg;
            double s = 0.0;
            for (int i = 0; i < m; ++i) s = fma((double)gj[i], Xv[i + (long)q * m], s);
            d.W[j + (long)q * d.ldw] = s;
        }
        __syncthreads();
    }
}

hipError_t launch_batched_wide(const void *desc, const int *order, int batch, int k, double tol, int nl, int *queue,
                               double *slabs, int grid, int nmax, int *rank, int *status, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = batched_lds_bytes(nl, nmax, k);
    hipLaunchKernelGGL(batched_wide_kernel, dim3(grid), dim3(BT_THREADS), lds, s,
                       static_cast<const BatchDesc *>(desc), order, batch, k, tol, nl, queue, slabs,
                       (long)batched_slab_doubles(nmax, k), nmax, rank, status);
    return hipGetLastError();
}

}  // namespace geninv
