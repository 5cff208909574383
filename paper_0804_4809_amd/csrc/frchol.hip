// Full-rank Cholesky factorization with column dropping (Section 2, Eq. (1);
// the Appendix's loop over k) on gfx950, blocked right-looking.
//
// The paper processes column k of A = G'G by subtracting the contribution of
// every column of L accepted so far, comparing the updated pivot with tol,
// and either keeping the column (sqrt and scale) or dropping it.  Here the
// columns are taken FR_NB at a time (a panel); when panel p starts, every
// earlier accepted column has already been subtracted from it:
//
//   1. panel factor (this file), one launch of one-wavefront workgroups,
//      each of which
//        - factors the diagonal block column by column with the paper's
//          strict "pivot > tol" test, keeping accepted columns only (the
//          block held in registers in a 2-D cyclic layout);
//        - for its own rows below the block, solves for the new L entries by
//          forward substitution against the accepted columns, in the same
//          column order as the paper, and writes them both compacted into L
//          and uncompacted (zero columns where a pivot was dropped) into the
//          n x FR_NB panel buffer Lp;
//      workgroup 0 writes the diagonal block of L, the pivot indices and the
//      new running rank rank_buf[p+1] = r0 + (accepted in this panel);
//   2. trailing update (an MFMA GEMM, gemm.hip): the lower triangle of
//      A[k1:n, k1:n] (k1 = k0 + w) loses Lp[k1:n, :] Lp[k1:n, :]', in place.
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
// itself, so that no workgroup waits for another.  Workgroup 0 then writes
// the block of L, the pivots and the new rank; every other workgroup also
// solves FR_TRS rows below the block against the accepted columns, four
// lanes per row, as it goes.
//
// The block is held in a 2-D cyclic layout: lane a + 8 b keeps
// v[r][c] = A(8 r + a, 8 c + b) for r >= c (register blocks with r < c lie
// wholly above the diagonal and are never touched).  For an accepted column
// J the lanes with b = J mod 8 publish column J (zero at rows <= J) in LDS
// before scaling, so that the round trip overlaps the reciprocal square
// root; every lane then reads the eight values for its row residue and the
// eight for its column residue, scales them, and applies the rank-one update
// to its registers on or past block J / 8.  A column costs two short LDS
// round trips and at most 36 fused multiply-adds per lane, where a
// row-per-lane layout needs a 63-way register broadcast.  Zeros at rows <= J
// keep finished columns and column J itself unchanged, so no lane tests its
// own indices.
//
// The rows below the block follow the paper's column-by-column update in the
// same loop: lane q of a row holds its entries at block columns 4t + q
// (t = 0..15), and at accepted column J
//   x_J <- x_J / L(J, J),  then  x_J' -= x_J L(J', J)  for J' > J.
// The new x_J is passed within the four lanes by a DPP quad broadcast, and
// L(J', J) comes from a second copy of column J in LDS laid out so that lane
// q reads its sixteen entries contiguously (zero at rows <= J, so the entries
// of finished columns are left alone).  Dropped columns leave the rows as
// they are.  At the end x holds the row of L at the accepted columns.

constexpr int FR_TRS = 16;             // rows per workgroup in the substitution
constexpr int FR_RB = FR_NB / 8;       // register blocks per dimension of the cyclic layout

// lane (4 (lane / 4) + Q)'s value of v, within each group of four lanes
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, Q * 0x55, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), Q * 0x55, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// LDS the factorization shares within the wavefront
struct FrShared {
    double colv[2][8][FR_RB];   // A(8 r + a, J) at [J & 1][a][r] before scaling, zero at rows <= J
    double coll[2][4][16];      // the same column at [J & 1][i mod 4][i / 4], for the row solve
    double dvs[FR_NB];          // pivot value of every column at its test
    int ccomp[FR_NB];           // compact index of block column j, or -1 if dropped
    int pcol[FR_NB];            // block column of compact column c
};

struct FrBlock {
    double v[FR_RB][FR_RB];   // v[r][c] = A(8 r + a, 8 c + b), then L; r >= c only
    double x[16];             // the lane's entries of its row below the block (block columns 4t + q)
    int acc;                  // accepted so far (uniform)
    double dv;                // pivot value of block column `lane`
    int cc;                   // compact index of block column `lane`, or -1
    int pc;                   // block column of compact column `lane`
};

// 1 / sqrt(d) for a positive normal d: the hardware estimate refined by two
// Newton steps (within an ulp or so; a much shorter dependency chain than a
// square root followed by a division)
__device__ __forceinline__ double rsqrt_refined(double d) {
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = __builtin_fma(0.5 * y, __builtin_fma(-d * y, y, 1.0), y);
    return y;
}

// Orders the LDS accesses of the wavefront's lanes (they execute in program
// order within one wavefront, so no wait for completion is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column J of the block: the paper's pivot test, then sqrt, scaling and the
// rank-one update of the later columns (every register index static), and,
// with `rows`, the same column's step of the row solve.  Every lane scales
// what it reads by the same factor, so its L(i, J) equals the owner's bit
// for bit.
template <int J>
__device__ __forceinline__ void fr_column(FrBlock &s, FrShared &sh, int a, int b, int q, int lane, int w, double tol,
                                          bool rows) {
    if (J >= w) return;
    constexpr int jr = J >> 3, jb = J & 7, r0 = jr & ~1, jt = J >> 2, jq = J & 3;
    const double d = lane_bcast(s.v[jr][jr], 9 * jb);   // current pivot of column J
    const bool keep = d > tol;                          // uniform
    s.dv = lane == J ? d : s.dv;
    s.cc = lane == J ? (keep ? s.acc : -1) : s.cc;
    if (!keep) return;
    double(*cv)[FR_RB] = sh.colv[J & 1];
    double(*cl)[16] = sh.coll[J & 1];
    if (b == jb) {
#pragma unroll
        for (int r = r0; r < FR_RB; r += 2) {
            const double e0 = (r >= jr && 8 * r + a > J) ? s.v[r][jr] : 0.0;
            const double e1 = 8 * (r + 1) + a > J ? s.v[r + 1][jr] : 0.0;
            *reinterpret_cast<double2 *>(&cv[a][r]) = double2{e0, e1};
            if (rows) {
                cl[(8 * r + a) & 3][(8 * r + a) >> 2] = e0;
                cl[(8 * r + 8 + a) & 3][(8 * r + 8 + a) >> 2] = e1;
            }
        }
    }
    wave_sync();
    double xi[FR_RB], xl[FR_RB];
#pragma unroll
    for (int r = r0; r < FR_RB; r += 2) {
        const double2 ti = *reinterpret_cast<const double2 *>(&cv[a][r]);
        const double2 tl = *reinterpret_cast<const double2 *>(&cv[b][r]);
        xi[r] = ti.x;
        xi[r + 1] = ti.y;
        xl[r] = tl.x;
        xl[r + 1] = tl.y;
    }
    double lc[16];
    if (rows) {
#pragma unroll
        for (int t = jt & ~1; t < 16; t += 2) {
            const double2 u = *reinterpret_cast<const double2 *>(&cl[q][t]);
            lc[t] = u.x;
            lc[t + 1] = u.y;
        }
    }
    const double y = rsqrt_refined(d);
    s.pc = lane == s.acc ? J : s.pc;
    if (b == jb) {
#pragma unroll
        for (int r = jr; r < FR_RB; ++r) {
            const int i = 8 * r + a;
            s.v[r][jr] = i > J ? s.v[r][jr] * y : (i == J ? d * y : s.v[r][jr]);
        }
    }
#pragma unroll
    for (int r = jr; r < FR_RB; ++r) {
        xi[r] *= y;
        xl[r] *= y;
    }
#pragma unroll
    for (int c = jr; c < FR_RB; ++c)
#pragma unroll
        for (int r = c; r < FR_RB; ++r) s.v[r][c] = __builtin_fma(-xi[r], xl[c], s.v[r][c]);
    if (rows) {
        // x_J / L(J, J) = x_J * y, from the lane holding column J of the row;
        // the entries at rows <= J of the copy are zero, so the update leaves
        // x_J and the finished entries alone
        const double xj = quad_bcast<jq>(s.x[jt] * y);
#pragma unroll
        for (int t = jt; t < 16; ++t) s.x[t] = __builtin_fma(-xj, lc[t] * y, s.x[t]);
        s.x[jt] = q == jq ? xj : s.x[jt];
    }
    wave_sync();
    ++s.acc;
}

template <int... J>
__device__ __forceinline__ void fr_factor(std::integer_sequence<int, J...>, FrBlock &s, FrShared &sh, int a, int b,
                                          int q, int lane, int w, double tol, bool rows) {
    (fr_column<J>(s, sh, a, b, q, lane, w, tol, rows), ...);
}

// P points at the panel: rows k0..n-1 of the panel's w columns (leading
// dimension ldp), A minus the contribution of every column accepted before
// the panel.
__global__ __launch_bounds__(64) void frchol_panel_kernel(const double *__restrict__ P, long ldp,
                                                          double *__restrict__ L, long ldl, int *rank_buf, int p,
                                                          int k0, int w, int n, const double *tolp, int *piv,
                                                          double *dvals, double *__restrict__ Lp, long ldlp) {
    __shared__ __align__(16) FrShared sh;

    const int lane = threadIdx.x;
    const int q = lane & 3;
    const int ra = lane & 7, cb = lane >> 3;   // row and column residue in the cyclic layout
    const int r0 = rank_buf[p];
    const double tol = *tolp;
    const bool rows = blockIdx.x > 0;         // uniform: this workgroup solves rows below the block
    const int irel = w + (int)(blockIdx.x - 1) * FR_TRS + (lane >> 2);
    const bool trs = rows && k0 + irel < n;

    FrBlock s;
    // this lane's entries of its row below the block (block column order),
    // in flight with the block's loads
#pragma unroll
    for (int t = 0; t < 16; ++t) s.x[t] = ld_or(P, irel + (long)(4 * t + q) * ldp, trs && 4 * t + q < w, 0.0);
    // the lower triangle of the block in the cyclic layout (zero above the
    // diagonal and past w)
#pragma unroll
    for (int r = 0; r < FR_RB; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            const int i = 8 * r + ra, j = 8 * c + cb;
            s.v[r][c] = ld_or(P, i + (long)j * ldp, i < w && j <= i, 0.0);
        }
    s.acc = 0;
    s.dv = 0.0;
    s.cc = -1;
    s.pc = 0;
    fr_factor(std::make_integer_sequence<int, FR_NB>{}, s, sh, ra, cb, q, lane, w, tol, rows);
    const int a = s.acc;
    sh.dvs[lane] = s.dv;
    sh.ccomp[lane] = s.cc;
    sh.pcol[lane] = s.pc;
    __syncthreads();

    if (!rows) {
        // diagonal block of L, pivots, pivot values, running rank
#pragma unroll
        for (int r = 0; r < FR_RB; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                const int i = 8 * r + ra, j = 8 * c + cb;
                const int cj = sh.ccomp[j];
                if (i < w && j <= i && cj >= 0) L[(k0 + i) + (long)(r0 + cj) * ldl] = s.v[r][c];
            }
        if (lane < w && dvals) dvals[k0 + lane] = sh.dvs[lane];
        if (lane < a && piv) piv[r0 + lane] = k0 + sh.pcol[lane];
        if (lane == 0) rank_buf[p + 1] = r0 + a;
        return;
    }
    if (!trs) return;
    // the row of L, compacted into L and uncompacted (zero where a column was
    // dropped) into the panel buffer Lp
    double *lrow = L + (k0 + irel) + (long)r0 * ldl;
    double *prow = Lp + (k0 + irel);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int j = 4 * t + q;
        if (j < w) {
            const int cj = sh.ccomp[j];
            if (cj >= 0) lrow[(long)cj * ldl] = s.x[t];
            prow[(long)j * ldlp] = cj >= 0 ? s.x[t] : 0.0;
        }
    }
}

hipError_t launch_frchol_panel(const double *P, long ldp, double *L, long ldl, int *rank_buf, int p, int k0, int w,
                               int n, const double *tol, int *piv, double *dvals, double *Lp, long ldlp,
                               hipStream_t s) {
    const int below = n - k0 - w;   // rows under the block
    dim3 grid(1 + (below + FR_TRS - 1) / FR_TRS);
    hipLaunchKernelGGL(frchol_panel_kernel, grid, dim3(64), 0, s, P, ldp, L, ldl, rank_buf, p, k0, w, n, tol, piv,
                       dvals, Lp, ldlp);
    return hipGetLastError();
}

}  // namespace geninv
