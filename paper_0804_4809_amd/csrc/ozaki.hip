// Error-free split products on the bfloat16 matrix cores of gfx950: the
// mixed-precision form of the Gram matrix A = G'G (Section 2, Eq. (1)) and of
// the chain's last product Y = P G' (Theorem 1).
//
// Operand slicing (the error-free transformation of Ozaki, Ogita, Oishi and
// Rump, Numer. Algorithms 2012): each row or column v of an operand gets an
// exponent e with max |v| < 2^e; v / 2^e in (-1, 1) is cut, most significant
// first, into `s` signed 8-bit integer slices by truncation toward zero.  A
// slice is an integer of magnitude <= 255, exact in bfloat16, and a product of
// two slices is an integer <= 255^2, exact in float32.
//
// Sliced product: C_ij = 2^(ea_i + eb_j) sum over slice pairs (t, u) of
// 2^(-8 (t+u+2)) (A_t B_u)_ij.  Each pair product runs on
// v_mfma_f32_16x16x32_bf16 in float32; after at most 256 values of k the
// partial sum (|.| <= 256 * 255^2 < 2^24) is still an exactly represented
// integer, so it is moved into a float64 total (scaled by the exact power of
// two of its pair) and the float32 accumulator restarts.  Every integer
// product is therefore exact and only the float64 totals round.
//
// Both operands are stored K-contiguous ("TN"): opA(i, k) = A_t[k + i lda],
// opB(k, j) = B_u[k + j ldb], planes `sa` / `sb` elements apart, with the K
// extent padded with zeros to a multiple of 64 by the slicing kernels.
#include "common.h"

namespace geninv {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// exponents: smallest e with max |x| < 2^e, 0 for an all-zero vector
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bound_exponent(double mx) {
    if (!(mx > 0.0)) return 0;
    int p;
    (void)frexp(mx, &p);   // mx = f 2^p, f in [0.5, 1)
    return p;
}

__global__ __launch_bounds__(256) void col_exponent_kernel(const double *X, long ldx, int rows, int cols, int *e) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    if (j >= cols) return;
    double mx = 0.0;
    const double *col = X + (long)j * ldx;
    for (int i = threadIdx.x; i < rows; i += 256) mx = fmax(mx, fabs(col[i]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) e[j] = bound_exponent(red[0]);
}

__global__ __launch_bounds__(256) void row_exponent_kernel(const double *X, long ldx, int rows, int cols, int *e) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    double mx = 0.0;
    for (int j = 0; j < cols; ++j) mx = fmax(mx, fabs(X[i + (long)j * ldx]));
    e[i] = bound_exponent(mx);
}

// the s slices of x / 2^e, most significant first
template <int S>
__device__ __forceinline__ void slice_value(double x, int e, __bf16 *out) {
    double r = ldexp(x, -e);
#pragma unroll
    for (int t = 0; t < S; ++t) {
        r *= 256.0;
        const double st = trunc(r);
        r -= st;
        out[t] = (__bf16)(float)st;
    }
}

// planes[t][i + j ldp] = slice t of X(i, j) with the column exponent e[j];
// rows rows..ldp-1 are written as zeros
template <int S>
__global__ __launch_bounds__(256) void slice_cols_kernel(const double *X, long ldx, int rows, int cols,
                                                         const int *e, __bf16 *planes, long ldp, long sp) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= ldp || j >= cols) return;
    __bf16 v[S];
    if (i < rows) {
        slice_value<S>(X[i + (long)j * ldx], e[j], v);
    } else {
#pragma unroll
        for (int t = 0; t < S; ++t) v[t] = (__bf16)0.0f;
    }
#pragma unroll
    for (int t = 0; t < S; ++t) planes[t * sp + i + (long)j * ldp] = v[t];
}

// transposed row slicing: planes[t][k + i ldp] = slice t of X(i, k) with the
// row exponent e[i]; k = cols..ldp-1 written as zeros.  32 x 32 tiles staged
// through LDS so that both the read (down columns of X) and the write (along
// rows of X) are contiguous.
template <int S>
__global__ __launch_bounds__(256) void slice_rows_t_kernel(const double *X, long ldx, int rows, int cols,
                                                           const int *e, __bf16 *planes, long ldp, long sp) {
    __shared__ double tile[32][33];
    const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int yy = ty; yy < 32; yy += 8) {
        const int i = i0 + tx, k = k0 + yy;
        tile[yy][tx] = (i < rows && k < cols) ? X[i + (long)k * ldx] : 0.0;
    }
    __syncthreads();
    for (int yy = ty; yy < 32; yy += 8) {
        const int i = i0 + yy, k = k0 + tx;
        if (i >= rows || k >= ldp) continue;
        __bf16 v[S];
        if (k < cols) {
            slice_value<S>(tile[tx][yy], e[i], v);
        } else {
#pragma unroll
            for (int t = 0; t < S; ++t) v[t] = (__bf16)0.0f;
        }
#pragma unroll
        for (int t = 0; t < S; ++t) planes[t * sp + k + (long)i * ldp] = v[t];
    }
}

// ---------------------------------------------------------------------------
// sliced GEMM
// ---------------------------------------------------------------------------
constexpr int SG_BM = 128, SG_BN = 128, SG_BK = 64;
constexpr int SG_WM = 4, SG_WN = 2;              // 8 wavefronts, each 32 x 64
constexpr int SG_LDK = SG_BK + 8;                // LDS row pitch (bf16), breaks bank conflicts
constexpr int SG_FLUSH = 256;                    // k values per exact float32 chunk

__global__ __launch_bounds__(512) void sliced_gemm_kernel(SlicedGemmArgs p) {
    constexpr int NT = 512;
    constexpr int TM = SG_BM / SG_WM, TN = SG_BN / SG_WN;   // 32 x 64
    constexpr int FM = TM / 16, FN = TN / 16;               // 2 x 4 blocks
    __shared__ __attribute__((aligned(16))) __bf16 As[2][SG_BM][SG_LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][SG_BN][SG_LDK];

    const int row0 = blockIdx.x * SG_BM, col0 = blockIdx.y * SG_BN;
    if (p.lower && col0 >= row0 + SG_BM) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % SG_WM, wn = wave / SG_WM;

    // global -> register staging: each thread moves two 16-byte chunks per operand
    uint4 ra[2], rb[2];
    auto gload = [&](const __bf16 *A, const __bf16 *B, int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + NT * q;
            const int r = c >> 3, kc = (c & 7) * 8;
            const int gi = row0 + r, gj = col0 + r;
            ra[q] = gi < p.M ? *reinterpret_cast<const uint4 *>(A + (long)gi * p.lda + k0 + kc) : uint4{0, 0, 0, 0};
            rb[q] = gj < p.N ? *reinterpret_cast<const uint4 *>(B + (long)gj * p.ldb + k0 + kc) : uint4{0, 0, 0, 0};
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + NT * q;
            const int r = c >> 3, kc = (c & 7) * 8;
            *reinterpret_cast<uint4 *>(&As[buf][r][kc]) = ra[q];
            *reinterpret_cast<uint4 *>(&Bs[buf][r][kc]) = rb[q];
        }
    };

    double tot[FM][FN][4];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) tot[a][b][v] = 0.0;

    const int nst = p.Kpad / SG_BK;
    constexpr int FLUSH_ST = SG_FLUSH / SG_BK;
    for (int pr = 0; pr < p.npairs; ++pr) {
        const __bf16 *A = p.A + (long)p.pt[pr] * p.sa;
        const __bf16 *B = p.B + (long)p.pu[pr] * p.sb;
        const double w = p.pw[pr];
        f4 acc[FM][FN];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        gload(A, B, 0);
        sstore(0);
        __syncthreads();
        for (int st = 0; st < nst; ++st) {
            const int buf = st & 1;
            const bool more = st + 1 < nst;
            if (more) gload(A, B, (st + 1) * SG_BK);
#pragma unroll
            for (int kk = 0; kk < SG_BK; kk += 32) {
                const int ko = kk + 8 * (lane >> 4);
                bf8 af[FM], bfr[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a)
                    af[a] = *reinterpret_cast<const bf8 *>(&As[buf][wm * TM + a * 16 + (lane & 15)][ko]);
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    bfr[b] = *reinterpret_cast<const bf8 *>(&Bs[buf][wn * TN + b * 16 + (lane & 15)][ko]);
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[b], af[a], acc[a][b], 0, 0, 0);
            }
            if ((st + 1) % FLUSH_ST == 0 || !more) {
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) tot[a][b][v] = fma(w, (double)acc[a][b][v], tot[a][b][v]);
                        acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
            if (more) sstore(buf ^ 1);
            __syncthreads();
        }
    }

    // result element (row, col): MFMA row index = column of C (4 (lane/16) + v),
    // MFMA column index = row of C (lane & 15)
#pragma unroll
    for (int a = 0; a < FM; ++a) {
        const int r = row0 + wm * TM + a * 16 + (lane & 15);
        if (r >= p.M) continue;
        const int er = p.ea[r];
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * TN + b * 16 + 4 * (lane >> 4) + v;
                if (c >= p.N || (p.lower && r < c)) continue;
                double *dst = p.C + r + (long)c * p.ldc;
                const double val = ldexp(tot[a][b][v], er + p.eb[c]);
                *dst = (p.beta != 0.0) ? val + p.beta * (*dst) : val;
            }
    }
}

hipError_t launch_col_exponents(const double *X, long ldx, int rows, int cols, int *e, hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_exponent_kernel, dim3(cols), dim3(256), 0, s, X, ldx, rows, cols, e);
    return hipGetLastError();
}

hipError_t launch_row_exponents(const double *X, long ldx, int rows, int cols, int *e, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(row_exponent_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, X, ldx, rows, cols, e);
    return hipGetLastError();
}

template <int S>
static hipError_t slice_cols_s(const double *X, long ldx, int rows, int cols, const int *e, __bf16 *planes, long ldp,
                               long sp, hipStream_t s) {
    dim3 grid((ldp + 255) / 256, cols);
    hipLaunchKernelGGL((slice_cols_kernel<S>), grid, dim3(256), 0, s, X, ldx, rows, cols, e, planes, ldp, sp);
    return hipGetLastError();
}

template <int S>
static hipError_t slice_rows_t_s(const double *X, long ldx, int rows, int cols, const int *e, __bf16 *planes,
                                 long ldp, long sp, hipStream_t s) {
    dim3 grid((rows + 31) / 32, (ldp + 31) / 32);
    hipLaunchKernelGGL((slice_rows_t_kernel<S>), grid, dim3(256), 0, s, X, ldx, rows, cols, e, planes, ldp, sp);
    return hipGetLastError();
}

hipError_t launch_slice_cols(const double *X, long ldx, int rows, int cols, const int *e, int nslices,
                             __bf16 *planes, long ldp, long sp, hipStream_t s) {
    if (rows < 0 || cols <= 0) return hipSuccess;
    switch (nslices) {
        case 1: return slice_cols_s<1>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 2: return slice_cols_s<2>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 3: return slice_cols_s<3>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 4: return slice_cols_s<4>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 5: return slice_cols_s<5>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 6: return slice_cols_s<6>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_slice_rows_t(const double *X, long ldx, int rows, int cols, const int *e, int nslices,
                               __bf16 *planes, long ldp, long sp, hipStream_t s) {
    if (rows <= 0 || cols < 0) return hipSuccess;
    switch (nslices) {
        case 1: return slice_rows_t_s<1>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 2: return slice_rows_t_s<2>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 3: return slice_rows_t_s<3>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 4: return slice_rows_t_s<4>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 5: return slice_rows_t_s<5>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        case 6: return slice_rows_t_s<6>(X, ldx, rows, cols, e, planes, ldp, sp, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sliced_gemm(const SlicedGemmArgs &a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    dim3 grid((a.M + SG_BM - 1) / SG_BM, (a.N + SG_BN - 1) / SG_BN);
    hipLaunchKernelGGL(sliced_gemm_kernel, grid, dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace geninv
