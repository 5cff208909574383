// Float64 products with few output columns and a long inner dimension,
// C (M x N) = alpha op(A) op(B) + beta C with A not transposed and N <= 16:
// the least-squares right-hand sides, W = Y F with Y = G^+ (Theorem 1
// applied to the k columns of F), and the like.  Such a product reads A
// (M x K) once and does 2 N flops per element read, so it is bound by HBM,
// not by the matrix cores; on MFMA tiles of 64 columns most of each tile
// would be padding.
//
// One thread owns one row of C and walks a chunk of K: A is read down its
// columns (consecutive rows per wavefront, eight loads in flight per
// thread), and op(B), transposed once into a K x NP row-major copy Bt (NP =
// N rounded up to a power of two, zero padded), is read at addresses that
// are uniform across the workgroup, so those loads go through the scalar
// unit.  Chunk s writes its partial sums to part[s]; the existing reduction
// kernel adds the chunks in a fixed order and applies alpha and beta.
#include "common.h"

namespace geninv {

constexpr int SK_ROWS = 256;   // rows of C per workgroup, one per thread
constexpr int SK_UNROLL = 8;   // loads of A in flight per thread

// Bt[k * NP + j] = op(B)(k, j) for j < N, zero for N <= j < NP
__global__ __launch_bounds__(256) void sk_transpose_kernel(const double *__restrict__ B, long ldb, int transB,
                                                           int K, int N, int NP, double *__restrict__ Bt) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)K * NP) return;
    const int k = (int)(e / NP), j = (int)(e % NP);
    double v = 0.0;
    if (j < N) v = transB ? B[j + (long)k * ldb] : B[k + (long)j * ldb];
    Bt[e] = v;
}

template <int NP>
__global__ __launch_bounds__(SK_ROWS) void sk_partial_kernel(const double *__restrict__ A, long lda,
                                                             const double *__restrict__ Bt, int M, int N, int K,
                                                             int kchunk, double *__restrict__ part, long strideP) {
    const int i = blockIdx.x * SK_ROWS + threadIdx.x;
    const int kb = blockIdx.y * kchunk;
    const int ke = min(K, kb + kchunk);
    double acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = 0.0;
    if (i < M) {
        const double *a = A + i;
        int k = kb;
        for (; k + SK_UNROLL <= ke; k += SK_UNROLL) {
            double av[SK_UNROLL];
#pragma unroll
            for (int u = 0; u < SK_UNROLL; ++u) av[u] = a[(long)(k + u) * lda];
#pragma unroll
            for (int u = 0; u < SK_UNROLL; ++u)
#pragma unroll
                for (int j = 0; j < NP; ++j) acc[j] = __builtin_fma(av[u], Bt[(long)(k + u) * NP + j], acc[j]);
        }
        for (; k < ke; ++k) {
            const double av = a[(long)k * lda];
#pragma unroll
            for (int j = 0; j < NP; ++j) acc[j] = __builtin_fma(av, Bt[(long)k * NP + j], acc[j]);
        }
        double *p = part + (long)blockIdx.y * strideP + i;
#pragma unroll
        for (int j = 0; j < NP; ++j)
            if (j < N) p[(long)j * M] = acc[j];
    }
}

int skinny_padded_width(int N) {
    int np = 1;
    while (np < N) np *= 2;
    return np;
}

// Bt needs K * skinny_padded_width(N) doubles, part S * M * N with
// S = ceil(K / kchunk); C = alpha * sum of the partials + beta * C.
hipError_t launch_skinny_gemm(const double *A, long lda, const double *B, long ldb, int transB, int M, int N, int K,
                              double alpha, double beta, double *C, long ldc, int kchunk, double *Bt, double *part,
                              hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (N > 16 || K <= 0 || kchunk <= 0) return hipErrorInvalidValue;
    const int NP = skinny_padded_width(N);
    const int S = (K + kchunk - 1) / kchunk;
    const long nt = (long)K * NP;
    hipLaunchKernelGGL(sk_transpose_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, B, ldb, transB, K,
                       N, NP, Bt);
    const dim3 grid((M + SK_ROWS - 1) / SK_ROWS, S);
    const long strideP = (long)M * N;
    switch (NP) {
    case 1: hipLaunchKernelGGL(sk_partial_kernel<1>, grid, dim3(SK_ROWS), 0, s, A, lda, Bt, M, N, K, kchunk, part, strideP); break;
    case 2: hipLaunchKernelGGL(sk_partial_kernel<2>, grid, dim3(SK_ROWS), 0, s, A, lda, Bt, M, N, K, kchunk, part, strideP); break;
    case 4: hipLaunchKernelGGL(sk_partial_kernel<4>, grid, dim3(SK_ROWS), 0, s, A, lda, Bt, M, N, K, kchunk, part, strideP); break;
    case 8: hipLaunchKernelGGL(sk_partial_kernel<8>, grid, dim3(SK_ROWS), 0, s, A, lda, Bt, M, N, K, kchunk, part, strideP); break;
    default: hipLaunchKernelGGL(sk_partial_kernel<16>, grid, dim3(SK_ROWS), 0, s, A, lda, Bt, M, N, K, kchunk, part, strideP); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_splitk_reduce(part, M, strideP, S, C, ldc, hdim(M), hdim(N), alpha, beta, GEMM_FULL, s);
}

}  // namespace geninv
