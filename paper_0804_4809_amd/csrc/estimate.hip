// Helpers of the mixed form's error estimate: random sign probe blocks and
// the squared Frobenius norms of a difference and of its reference.
#include "common.h"

#include <algorithm>

namespace geninv {

// Random sign probes for the error estimate: X(i, j) = +-1 from the top bit
// of splitmix64 (Steele, Lea and Flood, 2014) of (seed, i, j).
__global__ void probe_fill_kernel(double *X, long ldx, int rows, int cols, unsigned long long seed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= rows || j >= cols) return;
    unsigned long long z = seed + 0x9e3779b97f4a7c15ULL * (((unsigned long long)j << 32) + (unsigned)i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z ^= z >> 31;
    X[i + (long)j * ldx] = (z >> 63) ? 1.0 : -1.0;
}

hipError_t launch_probe_fill(double *X, long ldx, int rows, int cols, unsigned long long seed, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(probe_fill_kernel, dim3((rows + 255) / 256, cols), dim3(256), 0, s, X, ldx, rows, cols, seed);
    return hipGetLastError();
}

// out[0] += ||X - Y||_F^2, out[1] += ||Y||_F^2 over rows x cols (one atomic
// add per workgroup and sum)
__global__ __launch_bounds__(256) void diff_fro2_kernel(const double *X, long ldx, const double *Yp, long ldy,
                                                        int rows, int cols, double *out) {
    __shared__ double red[2][256];
    double d2 = 0.0, y2 = 0.0;
    const int j = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < rows; i += gridDim.x * 256) {
        const double y = Yp[i + (long)j * ldy];
        const double d = X[i + (long)j * ldx] - y;
        d2 = fma(d, d, d2);
        y2 = fma(y, y, y2);
    }
    red[0][threadIdx.x] = d2;
    red[1][threadIdx.x] = y2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(out, red[0][0]);
        atomicAdd(out + 1, red[1][0]);
    }
}

hipError_t launch_diff_fro2(const double *X, long ldx, const double *Yp, long ldy, int rows, int cols, double *out,
                            hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int bx = (int)std::min<long>(64, (rows + 255) / 256);
    hipLaunchKernelGGL(diff_fro2_kernel, dim3(bx, cols), dim3(256), 0, s, X, ldx, Yp, ldy, rows, cols, out);
    return hipGetLastError();
}

// out[0] = max_k diag[k] / min over accepted columns c < r of dvals[piv[c]]
// (the spread between the largest Gram diagonal and the smallest accepted
// pivot, a proxy for cond(L'L)); 0 when r = 0.  One workgroup.
__global__ __launch_bounds__(256) void kappa_kernel(const double *diag, const double *dvals, const int *piv,
                                                    const int *rank, int n, double *out) {
    __shared__ double mx[256], mn[256];
    const int r = *rank;
    double a = 0.0, b = INFINITY;
    for (int k = threadIdx.x; k < n; k += 256) a = fmax(a, diag[k]);
    for (int c = threadIdx.x; c < r; c += 256) b = fmin(b, dvals[piv[c]]);
    mx[threadIdx.x] = a;
    mn[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
            mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = r > 0 && mn[0] > 0.0 ? mx[0] / mn[0] : 0.0;
}

hipError_t launch_kappa(const double *diag, const double *dvals, const int *piv, const int *rank, int n, double *out,
                        hipStream_t s) {
    hipLaunchKernelGGL(kappa_kernel, dim3(1), dim3(256), 0, s, diag, dvals, piv, rank, n, out);
    return hipGetLastError();
}

}  // namespace geninv
