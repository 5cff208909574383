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

// ---- transposed A: C (M x N) = alpha A' B + beta C, A (K x M), B (K x N),
// N <= 16 -------------------------------------------------------------------
//
// The error estimate's G' V and G' (P V) (K = m rows of G, M = n columns).
// Each wavefront owns SKT_COLS consecutive columns of A and walks the rows
// of a chunk of K, one row per lane: every load of A covers 64 consecutive
// rows of one column (coalesced), and the four wavefronts of a workgroup
// (neighbouring column groups) load the same rows of B at the same time, so
// B is fetched about once per workgroup.  A lane's SKT_COLS x NP sums are
// reduced over the wavefront by a butterfly that halves the values each lane
// keeps at every step (63 exchanges for 64 values instead of 6 per value),
// and the chunks of K by the reduction kernel in a fixed order.

constexpr int SKT_COLS = 4;     // columns of A (rows of C) per wavefront
constexpr int SKT_UNROLL = 2;   // rows per lane per step (loads in flight: 2 (SKT_COLS + NP))

// cur[0..W) summed over the wavefront: at offset O a lane keeps half of its
// values (the upper half if lane & O) plus its partner's copy of that half;
// once one value is left the remaining offsets add it up.  Afterwards the
// lane holds the total of value index `base`.
template <int W, int O>
__device__ __forceinline__ void skt_butterfly(double *cur, int lane, int &base) {
    if constexpr (O >= 1) {
        if constexpr (W > 1) {
            constexpr int H = W / 2;
            const bool up = (lane & O) != 0;
#pragma unroll
            for (int t = 0; t < H; ++t) {
                const double send = up ? cur[t] : cur[t + H];
                const double keep = up ? cur[t + H] : cur[t];
                cur[t] = keep + __shfl_xor(send, O);
            }
            if (up) base += H;
            skt_butterfly<H, O / 2>(cur, lane, base);
        } else {
            cur[0] += __shfl_xor(cur[0], O);
            skt_butterfly<1, O / 2>(cur, lane, base);
        }
    }
}

template <int NP>
__global__ __launch_bounds__(256) void skt_partial_kernel(const double *__restrict__ A, long lda,
                                                          const double *__restrict__ B, long ldb, int M, int N, int K,
                                                          int kchunk, double *__restrict__ part, long strideP) {
    constexpr int V = SKT_COLS * NP;   // sums per lane, value index c NP + q
    static_assert(V <= 64 && (V & (V - 1)) == 0, "value count");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j0 = (blockIdx.x * 4 + wave) * SKT_COLS;
    const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);
    const double *acol[SKT_COLS];
#pragma unroll
    for (int c = 0; c < SKT_COLS; ++c) acol[c] = A + (long)min(j0 + c, M - 1) * lda;
    const double *bcol[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) bcol[q] = B + (long)min(q, N - 1) * ldb;
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
    for (int i0 = kb + lane; i0 < ke; i0 += SKT_UNROLL * 64) {
        double av[SKT_UNROLL][SKT_COLS], bv[SKT_UNROLL][NP];
#pragma unroll
        for (int u = 0; u < SKT_UNROLL; ++u) {
            const int i = i0 + u * 64;
            const bool ok = i < ke;
#pragma unroll
            for (int c = 0; c < SKT_COLS; ++c) av[u][c] = ld_or(acol[c], i, ok, 0.0);
#pragma unroll
            for (int q = 0; q < NP; ++q) bv[u][q] = ld_or(bcol[q], i, ok && q < N, 0.0);
        }
#pragma unroll
        for (int u = 0; u < SKT_UNROLL; ++u)
#pragma unroll
            for (int c = 0; c < SKT_COLS; ++c)
#pragma unroll
                for (int q = 0; q < NP; ++q) acc[c * NP + q] = __builtin_fma(av[u][c], bv[u][q], acc[c * NP + q]);
    }
    int base = 0;
    skt_butterfly<V, 32>(acc, lane, base);
    const int c = base / NP, q = base % NP;
    if ((lane & (64 / V - 1)) == 0 && j0 + c < M && q < N)
        part[(long)blockIdx.y * strideP + (j0 + c) + (long)q * M] = acc[0];
}

// part needs S * M * N doubles, S = ceil(K / kchunk); C = alpha * sum of the
// partials + beta * C.
hipError_t launch_skinny_gemm_t(const double *A, long lda, const double *B, long ldb, int M, int N, int K,
                                double alpha, double beta, double *C, long ldc, int kchunk, double *part,
                                hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (N > 16 || K <= 0 || kchunk <= 0) return hipErrorInvalidValue;
    const int NP = skinny_padded_width(N);
    const int S = (K + kchunk - 1) / kchunk;
    const dim3 grid((M + 4 * SKT_COLS - 1) / (4 * SKT_COLS), S);
    const long strideP = (long)M * N;
    switch (NP) {
    case 1: hipLaunchKernelGGL(skt_partial_kernel<1>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kchunk, part, strideP); break;
    case 2: hipLaunchKernelGGL(skt_partial_kernel<2>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kchunk, part, strideP); break;
    case 4: hipLaunchKernelGGL(skt_partial_kernel<4>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kchunk, part, strideP); break;
    case 8: hipLaunchKernelGGL(skt_partial_kernel<8>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kchunk, part, strideP); break;
    default: hipLaunchKernelGGL(skt_partial_kernel<16>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kchunk, part, strideP); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_splitk_reduce(part, M, strideP, S, C, ldc, hdim(M), hdim(N), alpha, beta, GEMM_FULL, s);
}

}  // namespace geninv
