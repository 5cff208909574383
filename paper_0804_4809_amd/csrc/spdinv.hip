// M = (L'L)^-1 (Theorem 1) on gfx950 by block Gauss-Jordan elimination.
//
// L'L is symmetric positive definite (L has full column rank r), so every
// pivot block met by Gauss-Jordan elimination without pivoting is a Schur
// complement of an SPD matrix and is itself SPD.  One elimination step on
// pivot block b (GJ_NB wide) of the r x r matrix B is
//
//   D       = B_bb^-1                        (pivot block, inverted in LDS)
//   R_j     = D B_bj          for j != b      (new pivot block row)
//   B_ij   -= B_ib R_j        for i, j != b   (rank-GJ_NB update)
//   B_ib    = -B_ib D         for i != b      (new pivot block column)
//   B_bj    = R_j,  B_bb = D
//
// and after the last block B holds B^-1.  Two launches per step: the panel
// kernel (D, R and a copy of the old block column, one workgroup per block
// column) and the update kernel (one workgroup per 64 x 64 tile), which reads
// only the staged panels so that tiles can be rewritten in place.  The
// 64 x 64 x 64 tile products run on v_mfma_f64_16x16x4f64.  The rank r is
// read from device memory; steps and tiles past r exit at once.
#include "common.h"

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

// In-LDS Gauss-Jordan inverse of the SPD block in X (column-major X[j][i]),
// w x w in the top-left corner and identity elsewhere, so that every thread
// updates a fixed set of elements without bounds tests.  Thread
// (lane, wave) owns row `lane`, columns wave, wave + 4, ...  Each step is one
// FMA per element (X -= column p * scaled row p), after which the owners of
// row p and column p overwrite them.  Returns false (uniformly) if a pivot is
// not positive.
__device__ bool gj_invert_block(double (*X)[GJ_LD], int w, double *rowp, double *colp) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    bool ok = true;
    for (int p = 0; p < w; ++p) {
        __syncthreads();
        const double pv = X[p][p];
        if (!(pv > 0.0)) ok = false;
        const double dinv = 1.0 / pv;
        if (tid < GJ_NB) {
            rowp[tid] = X[tid][p] * dinv;   // row p scaled by the inverse pivot
            colp[tid] = X[p][tid];          // column p
        }
        __syncthreads();
        const double cp = colp[lane];
        double v[GJ_NB / 4], rp[GJ_NB / 4];
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            v[q] = X[wave + 4 * q][lane];
            rp[q] = rowp[wave + 4 * q];
        }
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) X[wave + 4 * q][lane] = v[q] - cp * rp[q];
        if (lane == p) {
#pragma unroll
            for (int q = 0; q < GJ_NB / 4; ++q) X[wave + 4 * q][p] = rp[q];
        }
        if (wave == (p & 3)) X[p][lane] = lane == p ? dinv : -cp * dinv;
    }
    __syncthreads();
    return ok;
}

__global__ __launch_bounds__(256) void gj_panel_kernel(const double *__restrict__ B, long ldb, Dim rd, int b,
                                                       double *__restrict__ Dbuf, double *__restrict__ Rrow,
                                                       double *__restrict__ Ccol, long ldc, int *status) {
    __shared__ double X[GJ_NB][GJ_LD];
    __shared__ double Bl[GJ_NB][GJ_LD];
    __shared__ double rowp[GJ_NB], colp[GJ_NB];
    const int r = rd.get();
    const int nbk = (r + GJ_NB - 1) / GJ_NB;
    const int jb = blockIdx.x;
    if (b >= nbk || jb >= nbk) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wb = min(GJ_NB, r - b * GJ_NB);
    const int wj = min(GJ_NB, r - jb * GJ_NB);
    const long ob = (long)b * GJ_NB, oj = (long)jb * GJ_NB;

#pragma unroll
    for (int q = 0; q < GJ_NB / 4; ++q) {
        const int jc = wave + 4 * q;
        const bool in_b = lane < wb && jc < wb;
        X[jc][lane] = in_b ? B[(ob + lane) + (ob + jc) * ldb] : (lane == jc ? 1.0 : 0.0);
        // old block column (rows of block jb, columns of block b)
        if (lane < wj && jc < wb) Ccol[(oj + lane) + (long)jc * ldc] = B[(oj + lane) + (ob + jc) * ldb];
        // pivot block row restricted to the columns of block jb, zero padded
        Bl[jc][lane] = (jb != b && lane < wb && jc < wj) ? B[(ob + lane) + (oj + jc) * ldb] : 0.0;
    }
    const bool ok = gj_invert_block(X, wb, rowp, colp);
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
    if (b >= nbk || ib >= nbk || jb >= nbk) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wb = min(GJ_NB, r - b * GJ_NB);
    const int wi = min(GJ_NB, r - ib * GJ_NB);
    const int wj = min(GJ_NB, r - jb * GJ_NB);
    const long oi = (long)ib * GJ_NB, oj = (long)jb * GJ_NB;
    double *T = B + oi + oj * ldb;

    if (ib == b && jb == b) {
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            const int jc = wave + 4 * q;
            if (lane < wb && jc < wb) T[lane + (long)jc * ldb] = Dbuf[lane + (long)jc * GJ_NB];
        }
        return;
    }
    if (ib == b) {
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            const int jc = wave + 4 * q;
            if (lane < wb && jc < wj) T[lane + (long)jc * ldb] = Rrow[lane + (oj + jc) * GJ_NB];
        }
        return;
    }
    const bool newcol = jb == b;
    const int wr = newcol ? wb : wj;
#pragma unroll
    for (int q = 0; q < GJ_NB / 4; ++q) {
        const int kc = wave + 4 * q;
        // left factor: old block column rows of block ib (wi x wb), zero padded
        Xs[kc][lane] = (lane < wi && kc < wb) ? Ccol[(oi + lane) + (long)kc * ldc] : 0.0;
        // right factor: D (new block column) or R_jb, zero padded
        double y = 0.0;
        if (lane < wb && kc < wr) y = newcol ? Dbuf[lane + (long)kc * GJ_NB] : Rrow[lane + (oj + kc) * GJ_NB];
        Ys[kc][lane] = y;
    }
    __syncthreads();
    d4 acc[2][2];
    tile64_mfma(Xs, Ys, acc);
    const int wm = wave & 1, wn = wave >> 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * 32 + a * 16 + (lane & 15);
                const int col = wn * 32 + bb * 16 + (lane >> 4) + 4 * v;
                if (row < wi && col < wr) {
                    double *dst = T + row + (long)col * ldb;
                    *dst = newcol ? -acc[a][bb][v] : *dst - acc[a][bb][v];
                }
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

}  // namespace geninv
