// Kernels of the incremental factorization (Section 4, incremental
// learning): when p columns are appended to G, the full-rank Cholesky factor
// of the earlier columns stays as it is; the new rows of L solve a lower
// triangular system with the earlier pivot rows, L_P X = B_P, where
// L_P = L(piv, :) and B_P(c, i) = A(n_old + i, piv[c]) (the Appendix loop's
// update of a later column, written for all new columns at once), and the
// new columns' own decisions come from the full-rank Cholesky of their Schur
// complement.  Here: the gathers, the inverses of the 64 x 64 diagonal
// blocks of L_P (the solve is then blocked into MFMA products), and small
// copies.
#include "common.h"

namespace geninv {

// out(c, j) = X(idx[c], j), c < r, j < cols
__global__ void gather_rows_kernel(const double *X, long ldx, const int *idx, int r, int cols, double *out,
                                   long ldo) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (c < r && j < cols) out[c + (long)j * ldo] = X[idx[c] + (long)j * ldx];
}

hipError_t launch_gather_rows(const double *X, long ldx, const int *idx, int r, int cols, double *out, long ldo,
                              hipStream_t s) {
    if (r <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((r + 255) / 256, cols), dim3(256), 0, s, X, ldx, idx, r, cols, out,
                       ldo);
    return hipGetLastError();
}

// out(c, i) = X(row0 + i, idx[c]), c < r, i < p
__global__ void gather_cols_t_kernel(const double *X, long ldx, int row0, const int *idx, int r, int p, double *out,
                                     long ldo) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (c < r && i < p) out[c + (long)i * ldo] = X[row0 + i + (long)idx[c] * ldx];
}

hipError_t launch_gather_cols_t(const double *X, long ldx, int row0, const int *idx, int r, int p, double *out,
                                long ldo, hipStream_t s) {
    if (r <= 0 || p <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_cols_t_kernel, dim3((r + 255) / 256, p), dim3(256), 0, s, X, ldx, row0, idx, r, p, out,
                       ldo);
    return hipGetLastError();
}

// Y(i, c) = X(c, i), c < rows, i < cols (through 32 x 32 LDS tiles)
__global__ void transpose_kernel(const double *X, long ldx, double *Yp, long ldy, int rows, int cols) {
    __shared__ double t[32][33];
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    const int c0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
    for (int q = ty; q < 32; q += 8) {
        const int c = c0 + tx, i = i0 + q;
        if (c < rows && i < cols) t[q][tx] = X[c + (long)i * ldx];
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int i = i0 + tx, c = c0 + q;
        if (c < rows && i < cols) Yp[i + (long)c * ldy] = t[tx][q];
    }
}

hipError_t launch_transpose(const double *X, long ldx, double *Yp, long ldy, int rows, int cols, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_kernel, dim3((rows + 31) / 32, (cols + 31) / 32), dim3(32, 8), 0, s, X, ldx, Yp, ldy,
                       rows, cols);
    return hipGetLastError();
}

// dst[c] = src[c] + off, c < n
__global__ void offset_int_kernel(const int *src, int n, int off, int *dst) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) dst[c] = src[c] + off;
}

hipError_t launch_offset_int(const int *src, int n, int off, int *dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(offset_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, src, n, off, dst);
    return hipGetLastError();
}

// Inverse of diagonal block b (64 x 64, the last one possibly smaller) of the
// lower triangular T (r x r): Dinv + b * 64 * 64, column-major with ld 64,
// identity-padded.  One workgroup per block, thread j computes column j by
// forward substitution, D in LDS.
__global__ __launch_bounds__(64) void trinv64_kernel(const double *T, long ldt, int r, double *Dinv) {
    __shared__ double D[64][65];
    __shared__ double X[64][65];
    const int b = blockIdx.x, j = threadIdx.x;
    const int k0 = b * 64, nb = min(64, r - k0);
    for (int i = 0; i < 64; ++i) D[i][j] = (i < nb && j < nb) ? T[k0 + i + (long)(k0 + j) * ldt] : (i == j ? 1.0 : 0.0);
    __syncthreads();
    for (int i = 0; i < 64; ++i) {
        double v = 0.0;
        if (i == j) {
            v = 1.0 / D[i][i];
        } else if (i > j) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s = fma(D[i][k], X[k][j], s);
            v = -s / D[i][i];
        }
        X[i][j] = v;
    }
    for (int i = 0; i < 64; ++i) Dinv[(long)b * 4096 + i + 64 * j] = X[i][j];
}

hipError_t launch_trinv64(const double *T, long ldt, int r, double *Dinv, hipStream_t s) {
    if (r <= 0) return hipSuccess;
    hipLaunchKernelGGL(trinv64_kernel, dim3((r + 63) / 64), dim3(64), 0, s, T, ldt, r, Dinv);
    return hipGetLastError();
}

}  // namespace geninv
