// Full-rank Cholesky factorization with column dropping (Section 2, Eq. (1);
// the Appendix's loop over k) on gfx950, blocked left-looking.
//
// The paper processes column k of A = G'G by subtracting the contribution of
// every column of L accepted so far, comparing the updated pivot with tol,
// and either keeping the column (sqrt and scale) or dropping it.  Here the
// columns are taken FR_NB at a time (a panel):
//
//   1. panel update (an MFMA GEMM, split over K when the panel is tall and
//      narrow, gemm.hip): A[k0:n, k0:k0+w] -= L[k0:n, :r0] L[k0:k0+w, :r0]'
//      over the r0 columns accepted before the panel, written in place;
//   2. panel factor (this file), one launch, every workgroup:
//        - loads the updated diagonal block into LDS and factors it column by
//          column with the paper's strict "pivot > tol" test, keeping
//          accepted columns only (one wavefront, lane i owning row i);
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

// value of v held by lane l of the wavefront (l a compile-time constant in
// every use below)
__device__ __forceinline__ double lane_bcast(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

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

// Panel factor.  P points at the updated panel (the rows k0..n-1 of the
// panel's w columns, leading dimension ldp): A minus the contribution of the
// columns accepted before the panel.
__global__ __launch_bounds__(256) void frchol_panel_kernel(const double *__restrict__ P, long ldp,
                                                           double *__restrict__ L, long ldl, int *rank_buf,
                                                           int p, int k0, int w, int n, const double *tolp,
                                                           int *piv, double *dvals) {
    __shared__ double D[FR_NB][FR_NB + 1];   // D[j][i] = block entry (row i, column j)
    __shared__ double dpiv[FR_NB];           // updated pivot value of each block column
    __shared__ int outcol[FR_NB];            // L column of each accepted block column, -1 if dropped
    __shared__ double rdiag[FR_NB];          // 1 / L(j, j) of each accepted block column
    __shared__ int nacc;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r0 = rank_buf[p];
    const double tol = *tolp;

    // diagonal block (lower triangle) into LDS
#pragma unroll
    for (int q = 0; q < FR_NB / 4; ++q) {
        const int j = wave + 4 * q;
        if (lane < w && j < w && lane >= j) D[j][lane] = P[lane + (long)j * ldp];
    }
    __syncthreads();

    // one wavefront factors the block column by column; lane i owns row i of
    // the block in registers (fully unrolled, so every index is static).
    // The pivot and the scaled column are broadcast lane to lane
    // (v_readlane), without a round trip through memory.
    if (wave == 0) {
        double row[FR_NB];
#pragma unroll
        for (int l = 0; l < FR_NB; ++l) row[l] = (lane < w && l <= lane) ? D[l][lane] : 0.0;
        int acc = 0;
        double mydiag = 1.0;   // L(lane, lane) once column `lane` is accepted
#pragma unroll
        for (int j = 0; j < FR_NB; ++j) {
            if (j < w) {
                const double d = lane_bcast(row[j], j);   // current pivot of column j
                const bool keep = d > tol;                 // the same in every lane: uniform
                if (lane == 0) {
                    dpiv[j] = d;
                    outcol[j] = keep ? r0 + acc : -1;
                }
                if (keep) {
                    const double sq = sqrt(d);
                    const double lij = lane > j ? row[j] / sq : (lane == j ? sq : 0.0);
                    row[j] = lij;
                    if (lane == j) mydiag = sq;
#pragma unroll
                    for (int l0 = j + 1; l0 < FR_NB; l0 += 16) {
#pragma unroll
                        for (int l = l0; l < l0 + 16 && l < FR_NB; ++l) row[l] -= lij * lane_bcast(lij, l);
                        __builtin_amdgcn_sched_barrier(0);   // bound the scalar registers in flight
                    }
                    ++acc;
                }
            }
        }
        // factored block back to LDS (lower triangle), reciprocal pivots
#pragma unroll
        for (int l = 0; l < FR_NB; ++l)
            if (lane < w && l <= lane) D[l][lane] = row[l];
        if (lane < w) rdiag[lane] = 1.0 / mydiag;
        if (lane == 0) nacc = acc;
    }
    __syncthreads();

    // workgroup 0: diagonal block of L, pivots, pivot values, running rank
    if (blockIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < FR_NB / 4; ++q) {
            const int j = wave + 4 * q;
            if (j < w && lane < w && lane >= j) {
                const int c = outcol[j];
                if (c >= 0) L[(k0 + lane) + (long)c * ldl] = D[j][lane];
            }
        }
        if (tid < w) {
            if (dvals) dvals[k0 + tid] = dpiv[tid];
            if (piv && outcol[tid] >= 0) piv[outcol[tid]] = k0 + tid;
        }
        if (tid == 0) rank_buf[p + 1] = r0 + nacc;
    }

    // rows below the diagonal block: forward substitution, one row per thread,
    // in the paper's column order (division by the pivot taken as a product
    // with its reciprocal, computed once per column)
    const int irel = blockIdx.x * FR_ROWS + tid;
    if (irel < w || k0 + irel >= n) return;
    // keep the row loads below this point: hoisted into the block
    // factorization they would hold 64 more registers there and spill
    __builtin_amdgcn_sched_barrier(0);
    double x[FR_NB];
    // column base addresses are uniform (scalar registers); only the row
    // offset is per lane
#pragma unroll
    for (int j = 0; j < FR_NB; ++j) {
        const double *colj = P + (long)j * ldp;
        x[j] = j < w ? colj[irel] : 0.0;
    }
    double *lrow = L + (k0 + irel);
#pragma unroll
    for (int j = 0; j < FR_NB; ++j) {
        if (j < w) {
            const int c = outcol[j];
            if (c >= 0) {
                const double xj = x[j] * rdiag[j];
                lrow[(long)c * ldl] = xj;
                // groups of 16 broadcast reads, so that the compiler does not
                // hoist all 63 of them at once and spill x
#pragma unroll
                for (int l0 = j + 1; l0 < FR_NB; l0 += 16) {
#pragma unroll
                    for (int l = l0; l < l0 + 16 && l < FR_NB; ++l) x[l] -= xj * D[j][l];
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
}

hipError_t launch_frchol_panel(const double *P, long ldp, double *L, long ldl, int *rank_buf, int p, int k0, int w,
                               int n, const double *tol, int *piv, double *dvals, hipStream_t s) {
    const int rows = n - k0;
    dim3 grid((rows + FR_ROWS - 1) / FR_ROWS);
    hipLaunchKernelGGL(frchol_panel_kernel, grid, dim3(256), 0, s, P, ldp, L, ldl, rank_buf, p, k0, w, n, tol, piv,
                       dvals);
    return hipGetLastError();
}

}  // namespace geninv
