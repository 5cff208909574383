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
// only the staged panels so that tiles can be rewritten in place.  The rank r
// is read from device memory; steps and tiles past r exit at once.
#include "common.h"

namespace geninv {

constexpr int GJ_LD = GJ_NB + 1;

// in-LDS Gauss-Jordan inverse of the w x w block X (column-major X[j][i]);
// returns false (uniformly) if a pivot is not positive.
__device__ bool gj_invert_block(double (*X)[GJ_LD], int w, double *rowp, double *colp) {
    const int tid = threadIdx.x;
    bool ok = true;
    for (int p = 0; p < w; ++p) {
        __syncthreads();
        const double pv = X[p][p];
        if (!(pv > 0.0)) ok = false;
        const double dinv = 1.0 / pv;
        for (int t = tid; t < w; t += blockDim.x) {
            rowp[t] = X[t][p];   // row p, column t
            colp[t] = X[p][t];   // column p, row t
        }
        __syncthreads();
        for (int e = tid; e < w * w; e += blockDim.x) {
            const int i = e % w, j = e / w;
            double v;
            if (i == p && j == p) v = dinv;
            else if (i == p) v = rowp[j] * dinv;
            else if (j == p) v = -colp[i] * dinv;
            else v = X[j][i] - colp[i] * rowp[j] * dinv;
            X[j][i] = v;
        }
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
    const int wb = min(GJ_NB, r - b * GJ_NB);
    const int wj = min(GJ_NB, r - jb * GJ_NB);
    const long ob = (long)b * GJ_NB, oj = (long)jb * GJ_NB;

    for (int e = tid; e < wb * wb; e += 256) {
        const int i = e % wb, j = e / wb;
        X[j][i] = B[(ob + i) + (ob + j) * ldb];
    }
    // old block column (rows of block jb, columns of block b)
    for (int e = tid; e < wj * wb; e += 256) {
        const int i = e % wj, j = e / wj;
        Ccol[(oj + i) + (long)j * ldc] = B[(oj + i) + (ob + j) * ldb];
    }
    const bool ok = gj_invert_block(X, wb, rowp, colp);
    if (jb == b) {
        if (!ok && tid == 0) *status = ST_NOTSPD;
        for (int e = tid; e < wb * wb; e += 256) {
            const int i = e % wb, j = e / wb;
            Dbuf[i + (long)j * GJ_NB] = X[j][i];
        }
        return;
    }
    for (int e = tid; e < wb * wj; e += 256) {
        const int i = e % wb, j = e / wb;
        Bl[j][i] = B[(ob + i) + (oj + j) * ldb];
    }
    __syncthreads();
    // R = D * B_b,jb  (wb x wj)
    for (int e = tid; e < wb * wj; e += 256) {
        const int i = e % wb, j = e / wb;
        double s = 0.0;
        for (int k = 0; k < wb; ++k) s += X[k][i] * Bl[j][k];
        Rrow[i + (oj + j) * GJ_NB] = s;
    }
}

// tile (ib, jb) of the in-place update; products by LDS-staged FMA
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
    const int wb = min(GJ_NB, r - b * GJ_NB);
    const int wi = min(GJ_NB, r - ib * GJ_NB);
    const int wj = min(GJ_NB, r - jb * GJ_NB);
    const long oi = (long)ib * GJ_NB, oj = (long)jb * GJ_NB;
    double *T = B + oi + oj * ldb;

    if (ib == b && jb == b) {
        for (int e = tid; e < wb * wb; e += 256) {
            const int i = e % wb, j = e / wb;
            T[i + (long)j * ldb] = Dbuf[i + (long)j * GJ_NB];
        }
        return;
    }
    if (ib == b) {
        for (int e = tid; e < wb * wj; e += 256) {
            const int i = e % wb, j = e / wb;
            T[i + (long)j * ldb] = Rrow[i + (oj + j) * GJ_NB];
        }
        return;
    }
    // left factor: old block column rows of block ib (wi x wb)
    for (int e = tid; e < wi * wb; e += 256) {
        const int i = e % wi, k = e / wi;
        Xs[k][i] = Ccol[(oi + i) + (long)k * ldc];
    }
    // right factor: D (jb == b) or R_jb (wb x wj)
    const int wr = (jb == b) ? wb : wj;
    for (int e = tid; e < wb * wr; e += 256) {
        const int k = e % wb, j = e / wb;
        Ys[j][k] = (jb == b) ? Dbuf[k + (long)j * GJ_NB] : Rrow[k + (oj + j) * GJ_NB];
    }
    __syncthreads();
    const int i = tid & 63;
    const int j0 = tid >> 6;
    double accv[GJ_NB / 4];
#pragma unroll
    for (int q = 0; q < GJ_NB / 4; ++q) accv[q] = 0.0;
    if (i < wi) {
        for (int k = 0; k < wb; ++k) {
            const double xv = Xs[k][i];
#pragma unroll
            for (int q = 0; q < GJ_NB / 4; ++q) accv[q] += xv * Ys[j0 + 4 * q][k];
        }
#pragma unroll
        for (int q = 0; q < GJ_NB / 4; ++q) {
            const int j = j0 + 4 * q;
            if (j < wr) {
                double *dst = T + i + (long)j * ldb;
                if (jb == b) *dst = -accv[q];
                else *dst = *dst - accv[q];
            }
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
