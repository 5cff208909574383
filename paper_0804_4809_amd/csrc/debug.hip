// Debug support: fill a workspace with a quiet-NaN pattern so that a step
// reading memory no earlier step of the same call wrote shows up as NaN in
// the results (the pattern's 64-bit words are quiet NaNs).
#include "common.h"

namespace geninv {

__global__ void poison_kernel(unsigned long long *p, size_t n, unsigned long long v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_poison(void *p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 8;
    if (n == 0) return hipSuccess;
    if (reinterpret_cast<uintptr_t>(p) & 7) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)std::min<size_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(poison_kernel, dim3(blocks), dim3(256), 0, s, static_cast<unsigned long long *>(p), n,
                       0x7ff8dead0000beefull);
    return hipGetLastError();
}

}  // namespace geninv
