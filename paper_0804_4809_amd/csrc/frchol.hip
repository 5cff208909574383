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
//   2. panel factor (this file), one launch of one-wavefront workgroups,
//      each of which
//        - factors the updated diagonal block column by column with the
//          paper's strict "pivot > tol" test, keeping accepted columns only
//          (lane i owning row i in registers);
//        - for its own rows below the block, solves for the new L entries by
//          forward substitution against the accepted columns, in the same
//          column order as the paper;
//      workgroup 0 writes the diagonal block of L, the pivot indices and the
//      new running rank rank_buf[p+1] = r0 + (accepted in this panel).
//
// Accepted columns are written compacted (column r0, r0+1, ...), so L comes
// out n x r with zeros above each column's pivot row.  The running rank lives
// in device memory: rank_buf[p] is read by panel p and rank_buf[p+1] written,
// so no kernel reads a value another workgroup of the same launch writes.
#include "common.h"

#include <utility>

namespace geninv {


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

// ---- panel factor ---------------------------------------------------------
//
// Every workgroup is one wavefront.  Each one factors the diagonal block
// itself (lane i owning row i in registers, the pivot and the scaled column
// broadcast lane to lane with v_readlane), so that no workgroup waits for
// another.  Workgroup 0 then writes the block of L, the pivots and the new
// rank; every other workgroup solves FR_TRS rows below the block against the
// accepted columns, four lanes per row.
//
// The substitution runs over the accepted columns only, renumbered 0..a-1 in
// the paper's column order: for row x of the panel restricted to the accepted
// columns and T the a x a lower triangle of the block at the pivot rows,
//   x_c <- x_c / T_cc,  then  x_c' -= x_c T_c'c  for c' > c,
// which is the paper's column-by-column update of these rows.  Lane q of a
// row holds columns c = 4t + q (t = 0..15); the new x_c is passed within the
// four lanes by a DPP quad broadcast, and T is read from LDS, laid out so that
// lane q reads its own 16 entries of a column contiguously.

constexpr int FR_TRS = 16;             // rows per workgroup in the substitution
constexpr int FR_TSEG = 18;            // T row: 4 segments of 18 doubles (16 used): 16-byte aligned, banks spread
constexpr int FR_TLD = 4 * FR_TSEG;
constexpr int FR_BC = 16;              // broadcasts in flight per group in the block factorization
constexpr int FR_CH = 8;               // substitution columns per uniform chunk

// lane (4 (lane / 4) + Q)'s value of v, within each group of four lanes
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, Q * 0x55, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), Q * 0x55, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

struct FrBlock {
    double row[FR_NB];    // row `lane` of the block (lower triangle), then of L
    int acc;              // accepted so far (uniform)
    double mydiag;        // L(lane, lane) if column `lane` is accepted, else 1
    double mypiv;         // updated pivot value of column `lane`
    int myc;              // compact index of column `lane` if accepted, else -1
};

// Column J of the block: the paper's pivot test, then sqrt, scaling and the
// rank-one update of the later columns (every index static after expansion).
template <int J>
__device__ __forceinline__ void fr_column(FrBlock &s, int lane, int w, double tol) {
    if (J >= w) return;
    const double d = lane_bcast(s.row[J], J);   // current pivot of column J
    const bool keep = d > tol;                   // uniform
    if (lane == J) {
        s.mypiv = d;
        s.myc = keep ? s.acc : -1;
    }
    if (!keep) return;
    const double sq = sqrt(d);
    const double lij = lane > J ? s.row[J] / sq : (lane == J ? sq : 0.0);
    s.row[J] = lij;
    if (lane == J) s.mydiag = sq;
#pragma unroll
    for (int g = (J + 1) / FR_BC; g < FR_NB / FR_BC; ++g) {
        // FR_BC broadcasts into distinct scalar registers, then the FMAs
        double bc[FR_BC];
#pragma unroll
        for (int e = 0; e < FR_BC; ++e)
            if (g * FR_BC + e > J) bc[e] = lane_bcast(lij, g * FR_BC + e);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < FR_BC; ++e)
            if (g * FR_BC + e > J) s.row[g * FR_BC + e] -= lij * bc[e];
        __builtin_amdgcn_sched_barrier(0);
    }
    ++s.acc;
}

template <int... J>
__device__ __forceinline__ void fr_factor(std::integer_sequence<int, J...>, FrBlock &s, int lane, int w,
                                          double tol) {
    (fr_column<J>(s, lane, w, tol), ...);
}

// Compact column J of the substitution (branch-free; J >= a contributes 0).
template <int J>
__device__ __forceinline__ void trs_column(double (&x)[16], const double (&rd)[16], int q, int a, const double *tq) {
    const double xj0 = quad_bcast<J & 3>(x[J >> 2] * rd[J >> 2]);
    const double xj = J < a ? xj0 : 0.0;
    const double upd = x[J >> 2] - xj * tq[J * FR_TLD + (J >> 2)];
    x[J >> 2] = q == (J & 3) ? xj : upd;
#pragma unroll
    for (int t = (J >> 2) + 1; t < 16; ++t) x[t] -= xj * tq[J * FR_TLD + t];
}

template <int G, int... E>
__device__ __forceinline__ void trs_chunk(std::integer_sequence<int, E...>, double (&x)[16], const double (&rd)[16],
                                          int q, int a, const double *tq) {
    if (G * FR_CH >= a) return;   // uniform
    (trs_column<G * FR_CH + E>(x, rd, q, a, tq), ...);
}

template <int... G>
__device__ __forceinline__ void trs_solve(std::integer_sequence<int, G...>, double (&x)[16], const double (&rd)[16],
                                          int q, int a, const double *tq) {
    (trs_chunk<G>(std::make_integer_sequence<int, FR_CH>{}, x, rd, q, a, tq), ...);
}

// P points at the updated panel: rows k0..n-1 of the panel's w columns
// (leading dimension ldp), A minus the contribution of the columns accepted
// before the panel.
__global__ __launch_bounds__(64) void frchol_panel_kernel(const double *__restrict__ P, long ldp,
                                                          double *__restrict__ L, long ldl, int *rank_buf, int p,
                                                          int k0, int w, int n, const double *tolp, int *piv,
                                                          double *dvals) {
    __shared__ __align__(16) double T[FR_NB][FR_TLD];   // T[c][seg(c')] = L(pivot row of c', c), 0 unless c' > c
    __shared__ double S[FR_TRS][FR_NB + 1];             // row staging for the renumbering of the columns
    __shared__ double rdc[FR_NB];                       // 1 / L(pivot row of c, c)
    __shared__ int pcol[FR_NB];                         // block column of compact column c

    const int lane = threadIdx.x;
    const int q = lane & 3;
    const int r0 = rank_buf[p];
    const double tol = *tolp;
    const int irel = w + (int)(blockIdx.x - 1) * FR_TRS + (lane >> 2);
    const bool trs = blockIdx.x > 0 && k0 + irel < n;

    // this lane's entries of its row below the block (block column order),
    // in flight during the factorization
    double x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = ld_or(P, irel + (long)(4 * t + q) * ldp, trs && 4 * t + q < w, 0.0);

    FrBlock s;
#pragma unroll
    for (int l = 0; l < FR_NB; ++l) s.row[l] = ld_or(P, lane + (long)l * ldp, lane < w && l <= lane, 0.0);
    s.acc = 0;
    s.mydiag = 1.0;
    s.mypiv = 0.0;
    s.myc = -1;
    if (blockIdx.x > 0) {
        // zero T, so that the columns of the last chunk past a read zeros
        double *tf = &T[0][0];
#pragma unroll
        for (int e = 0; e < FR_NB * FR_TLD / 64; ++e) tf[e * 64 + lane] = 0.0;
    }
    fr_factor(std::make_integer_sequence<int, FR_NB>{}, s, lane, w, tol);
    const int a = s.acc;

    if (blockIdx.x == 0) {
        // diagonal block of L, pivots, pivot values, running rank
        if (lane < w) {
#pragma unroll
            for (int j = 0; j < FR_NB; ++j) {
                const int cj = __builtin_amdgcn_readlane(s.myc, j);   // uniform
                if (cj >= 0 && j <= lane) L[(k0 + lane) + (long)(r0 + cj) * ldl] = s.row[j];
            }
            if (dvals) dvals[k0 + lane] = s.mypiv;
            if (piv && s.myc >= 0) piv[r0 + s.myc] = k0 + lane;
        }
        if (lane == 0) rank_buf[p + 1] = r0 + a;
        return;
    }

    // compact triangle T and the reciprocal pivots, from the registers
#pragma unroll
    for (int j = 0; j < FR_NB; ++j) {
        const int cj = __builtin_amdgcn_readlane(s.myc, j);
        if (cj >= 0 && s.myc >= 0) T[cj][FR_TSEG * (s.myc & 3) + (s.myc >> 2)] = lane > j ? s.row[j] : 0.0;
    }
    if (s.myc >= 0) {
        rdc[s.myc] = 1.0 / s.mydiag;
        pcol[s.myc] = lane;
    }
    // renumber the row's entries to compact column order through LDS
    const int rl = lane >> 2;
    if (trs) {
#pragma unroll
        for (int t = 0; t < 16; ++t)
            if (4 * t + q < w) S[rl][4 * t + q] = x[t];
    }
    __syncthreads();
    if (!trs) return;
    double rd[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int c = 4 * t + q;
        x[t] = c < a ? S[rl][pcol[c]] : 0.0;
        rd[t] = c < a ? rdc[c] : 0.0;
    }
    trs_solve(std::make_integer_sequence<int, FR_NB / FR_CH>{}, x, rd, q, a, &T[0][FR_TSEG * q]);
    double *lrow = L + (k0 + irel) + (long)r0 * ldl;
#pragma unroll
    for (int t = 0; t < 16; ++t)
        if (4 * t + q < a) lrow[(long)(4 * t + q) * ldl] = x[t];
}

hipError_t launch_frchol_panel(const double *P, long ldp, double *L, long ldl, int *rank_buf, int p, int k0, int w,
                               int n, const double *tol, int *piv, double *dvals, hipStream_t s) {
    const int below = n - k0 - w;   // rows under the block
    dim3 grid(1 + (below + FR_TRS - 1) / FR_TRS);
    hipLaunchKernelGGL(frchol_panel_kernel, grid, dim3(64), 0, s, P, ldp, L, ldl, rank_buf, p, k0, w, n, tol, piv,
                       dvals);
    return hipGetLastError();
}

}  // namespace geninv
