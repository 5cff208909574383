// Full-rank Cholesky factorization with column dropping (Section 2, Eq. (1);
// the Appendix's loop over k) on gfx950, blocked left-looking.
//
// The paper processes column k of A = G'G by subtracting the contribution of
// every column of L accepted so far, comparing the updated pivot with tol,
// and either keeping the column (sqrt and scale) or dropping it.  Here the
// columns are taken FR_NB at a time (a panel):
//
//   1. panel update (a split-K MFMA GEMM, gemm.hip):
//        part_s = L[k0:n, slice_s] * L[k0:k0+w, slice_s]'
//      over the r0 columns accepted before the panel;
//   2. panel factor (this file), one launch, every workgroup:
//        - forms the updated diagonal block  A[k0:k0+w, k0:k0+w] - sum_s part_s
//          in LDS and factors it column by column with the paper's strict
//          "pivot > tol" test, keeping accepted columns only;
//        - for its own rows below the block, solves for the new L entries by
//          forward substitution against the accepted columns, in the same
//          column order as the paper;
//      workgroup 0 also writes the diagonal block of L, the pivot indices and
//      the new running rank rank_buf[p+1] = r0 + (accepted in this panel).
//
// Accepted columns are written compacted (column r0, r0+1, ...), so L comes
// out n x r with zeros above each column's pivot row.  The running rank lives
// in device memory: rank_buf[p] is read by panel p and rank_buf[p+1] written,
// so no kernel reads a value another workgroup of the same launch writes.
#include "common.h"

namespace geninv {

constexpr int FR_ROWS = 256;   // rows per workgroup in the panel factor (one per thread)

// tol = user_tol if > 0, else 1e-9 * min{A_kk > 0} (Appendix); +Inf when A has
// no positive diagonal (every pivot test then fails: r = 0).  A non-finite
// diagonal means G (or its Gram matrix) holds Inf/NaN: status is set and the
// threshold is +Inf, so the factorization keeps nothing.
__global__ __launch_bounds__(256) void tol_kernel(const double *A, long lda, int n, double user_tol,
                                                  double *tol_out, int *status) {
    __shared__ double smin[256];
    __shared__ int sbad[256];
    const int tid = threadIdx.x;
    double mn = __builtin_huge_val();
    int bad = 0;
    for (int k = tid; k < n; k += 256) {
        const double a = A[k + (long)k * lda];
        if (!__builtin_isfinite(a)) bad = 1;
        else if (a > 0.0 && a < mn) mn = a;
    }
    smin[tid] = mn;
    sbad[tid] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            smin[tid] = fmin(smin[tid], smin[tid + s]);
            sbad[tid] |= sbad[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double t;
        if (sbad[0]) {
            *status = ST_NONFINITE;
            t = __builtin_huge_val();
        } else if (user_tol > 0.0) {
            t = user_tol;
        } else {
            t = (smin[0] == __builtin_huge_val()) ? __builtin_huge_val() : smin[0] * 1e-9;
        }
        *tol_out = t;
    }
}

hipError_t launch_tol(const double *A, long lda, int n, double user_tol, double *tol_out, int *status,
                      hipStream_t s) {
    hipLaunchKernelGGL(tol_kernel, dim3(1), dim3(256), 0, s, A, lda, n, user_tol, tol_out, status);
    return hipGetLastError();
}

// Panel factor.  part holds S split-K partial products (S may be 0), laid out
// part[s*strideP + i + j*ldp] for panel-relative row i and panel column j.
__global__ __launch_bounds__(256) void frchol_panel_kernel(const double *__restrict__ A, long lda,
                                                           const double *__restrict__ part, long ldp,
                                                           long strideP, int S, double *__restrict__ L,
                                                           long ldl, int *rank_buf, int p, int k0, int w,
                                                           int n, const double *tolp, int *piv,
                                                           double *dvals) {
    __shared__ double D[FR_NB][FR_NB + 1];   // D[j][i] = block entry (row i, column j)
    __shared__ double dpiv[FR_NB];           // updated pivot value of each block column
    __shared__ int outcol[FR_NB];            // L column of each accepted block column, -1 if dropped

    const int tid = threadIdx.x;
    const int r0 = rank_buf[p];
    const double tol = *tolp;

    // 1. updated diagonal block (lower triangle)
    for (int e = tid; e < w * w; e += 256) {
        const int i = e % w, j = e / w;
        if (i >= j) {
            double v = A[(k0 + i) + (long)(k0 + j) * lda];
            for (int s = 0; s < S; ++s) v -= part[s * strideP + i + (long)j * ldp];
            D[j][i] = v;
        }
    }
    __syncthreads();

    // 2. column by column: strict test against tol, sqrt, scale, update the rest
    int acc = 0;
    for (int j = 0; j < w; ++j) {
        const double d = D[j][j];
        const bool keep = d > tol;          // same LDS value in every thread: uniform
        if (tid == 0) {
            dpiv[j] = d;
            outcol[j] = keep ? r0 + acc : -1;
        }
        __syncthreads();
        if (keep) {
            const double sq = sqrt(d);
            for (int i = j + 1 + tid; i < w; i += 256) D[j][i] = D[j][i] / sq;
            if (tid == 0) D[j][j] = sq;
            __syncthreads();
            const int t = w - j - 1;
            for (int e = tid; e < t * t; e += 256) {
                const int i = j + 1 + e % t, l = j + 1 + e / t;
                if (i >= l) D[l][i] -= D[j][i] * D[j][l];
            }
            __syncthreads();
            ++acc;
        }
    }

    // 3. workgroup 0: diagonal block of L, pivots, pivot values, running rank
    if (blockIdx.x == 0) {
        for (int e = tid; e < w * w; e += 256) {
            const int i = e % w, j = e / w;
            const int c = outcol[j];
            if (c >= 0 && i >= j) L[(k0 + i) + (long)c * ldl] = D[j][i];
        }
        for (int j = tid; j < w; j += 256) {
            if (dvals) dvals[k0 + j] = dpiv[j];
            if (piv && outcol[j] >= 0) piv[outcol[j]] = k0 + j;
        }
        if (tid == 0) rank_buf[p + 1] = r0 + acc;
    }

    // 4. rows below the diagonal block: forward substitution, one row per thread
    const int irel = blockIdx.x * FR_ROWS + tid;
    if (irel < w || k0 + irel >= n) return;
    double x[FR_NB];
    const double *arow = A + (k0 + irel) + (long)k0 * lda;
#pragma unroll
    for (int j = 0; j < FR_NB; ++j) {
        double v = 0.0;
        if (j < w) {
            v = arow[(long)j * lda];
            for (int s = 0; s < S; ++s) v -= part[s * strideP + irel + (long)j * ldp];
        }
        x[j] = v;
    }
    double *lrow = L + (k0 + irel);
#pragma unroll
    for (int j = 0; j < FR_NB; ++j) {
        if (j < w) {
            const int c = outcol[j];
            if (c >= 0) {
                const double xj = x[j] / D[j][j];
                lrow[(long)c * ldl] = xj;
#pragma unroll
                for (int l = j + 1; l < FR_NB; ++l) x[l] -= xj * D[j][l];
            }
        }
    }
}

hipError_t launch_frchol_panel(const double *A, long lda, const double *part, long ldp, long strideP, int S,
                               double *L, long ldl, int *rank_buf, int p, int k0, int w, int n,
                               const double *tol, int *piv, double *dvals, hipStream_t s) {
    const int rows = n - k0;
    dim3 grid((rows + FR_ROWS - 1) / FR_ROWS);
    hipLaunchKernelGGL(frchol_panel_kernel, grid, dim3(256), 0, s, A, lda, part, ldp, strideP, S, L, ldl,
                       rank_buf, p, k0, w, n, tol, piv, dvals);
    return hipGetLastError();
}

}  // namespace geninv
