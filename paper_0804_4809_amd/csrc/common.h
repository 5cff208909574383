// Internal declarations shared by the libgeninv HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace geninv {

// A matrix dimension that is either fixed on the host or read from device
// memory at kernel start (the rank r is only known on the device, so the
// kernels that depend on it are launched for an upper bound and read the
// actual value themselves; no host read-back is needed between steps).
struct Dim {
    int host;          // value used when dev == nullptr, and the launch upper bound
    const int *dev;    // optional device location of the actual value (<= host)
    __device__ __forceinline__ int get() const { return dev ? *dev : host; }
};

static inline Dim hdim(int v) { return Dim{v, nullptr}; }

// ---- direct global -> LDS loads (global_load_lds_dwordx4) ------------------
// one wavefront-wide direct load: 16 bytes per lane from g into LDS at
// l + 16 * lane (l uniform across the wavefront)
__device__ __forceinline__ void lds_load16(const void *g, void *l) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 16, 0, 0);
}

// wait until at most N of this wavefront's vector memory loads are pending
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// workgroup barrier for the stage buffers: this wavefront's LDS reads have
// returned, then s_barrier.  Unlike __syncthreads() it does not wait for
// every outstanding vector load, so direct loads of later stages stay in
// flight; each wavefront waits for the loads the next stage reads itself.
__device__ __forceinline__ void stage_barrier() {
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// p[i] if ok, else pad, with an unconditional load (the address falls back to
// p[0], which must be readable): loads written this way carry no branch, so a
// loop of them is issued back to back instead of one load and wait at a time.
__device__ __forceinline__ double ld_or(const double *p, long i, bool ok, double pad) {
    const double v = p[ok ? i : 0];
    return ok ? v : pad;
}
static inline Dim ddim(int bound, const int *p) { return Dim{bound, p}; }

// Output modes of the GEMM epilogue.
enum GemmUplo { GEMM_FULL = 0, GEMM_LOWER = 1 };

struct GemmArgs {
    const double *A; long lda; int transA;
    const double *B; long ldb; int transB;
    double *C; long ldc;
    Dim M, N, K;
    double alpha, beta;
    int uplo;          // GemmUplo; GEMM_LOWER skips tiles above the diagonal and elements with row < col
    int splitk;        // > 1: gridDim.z slices of K, raw partial sums written to C + z*strideC
    long strideC;
    int onelevel;      // 128-tile kernel: one running sum over K instead of the two-level sum
};

// Sliced (error-free split) GEMM on bfloat16 matrix cores, ozaki.hip.
constexpr int SG_MAX_S = 4;     // slices per operand (registers of the class loop)
struct SlicedGemmArgs {
    const __bf16 *A; long lda; long sa;   // opA(i, k) = A[t sa + k + i lda]
    const __bf16 *B; long ldb; long sb;   // opB(k, j) = B[u sb + k + j ldb]
    const int *ea; const int *eb;         // row exponents of opA, column exponents of opB
    double *C; long ldc;
    int M, N, Kpad;                       // Kpad: multiple of 64, zero padded in the planes
    int S;                                // slices of both operands
    int nclass;                           // pairs formed: weight classes t + u < nclass (2 S - 1: every pair)
    int lower;
    double beta;
    int splitk;                           // > 1: raw scaled partial sums to C + z strideC
    long strideC;
};

// Device status word values (match geninv_status).
enum { ST_OK = 0, ST_NONFINITE = -4, ST_NOTSPD = -5 };

// ---- launchers (kernels.hip) -------------------------------------------------
hipError_t launch_dgemm(const GemmArgs &a, hipStream_t s);
long gemm_tiles(const GemmArgs &a, int bm);   // workgroups a launch would use with bm x bm tiles
int choose_splits(long tiles, int K, int maxS); // split-K factor for `tiles` 128 x 128 tiles of depth K
int fill_splits(long tiles, int K, int maxS);   // the same, restricted to launches of >= 256 workgroups (0: none)
hipError_t launch_splitk_reduce(const double *part, long ldp, long strideP, int S, double *C, long ldc,
                                Dim M, Dim N, double alpha, double beta, int uplo, hipStream_t s);
hipError_t launch_fill(double *X, long ldx, int rows, int cols, double v, hipStream_t s);
hipError_t launch_fill_int(int *x, int n, int v, hipStream_t s);
hipError_t launch_copy(const double *X, long ldx, double *Yp, long ldy, Dim rows, Dim cols, hipStream_t s);
hipError_t launch_mirror_lower(double *X, long ldx, Dim n, hipStream_t s);
hipError_t launch_axpby(const double *X, long ldx, double *Yp, long ldy, Dim rows, Dim cols, double a, double b,
                        hipStream_t s);   // Y = a X + b Y
hipError_t launch_transpose(const double *X, long ldx, double *Yp, long ldy, int rows, int cols, hipStream_t s);
hipError_t launch_probe_fill(double *X, long ldx, int rows, int cols, unsigned long long seed, hipStream_t s);
hipError_t launch_diff_fro2(const double *X, long ldx, const double *Yp, long ldy, int rows, int cols, double *out,
                            hipStream_t s);   // out[0] += ||X - Y||_F^2, out[1] += ||Y||_F^2
hipError_t launch_kappa(const double *diag, const double *dvals, const int *piv, const int *rank, int n, double *out,
                        hipStream_t s);  // out[0] = max diag / min accepted pivot

// full-rank Cholesky (frchol.hip)
constexpr int FR_NB = 64;          // panel width
hipError_t launch_tol(const double *A, long lda, int n, double user_tol, double *tol_out, int *status,
                      hipStream_t s);
hipError_t launch_frchol_panel(const double *P, long ldp, double *L, long ldl, int *rank_buf, int p, int k0,
                               int w, int n, const double *tol, int *piv, double *dvals, double *Lp, long ldlp,
                               hipStream_t s);

// SPD inverse by block Gauss-Jordan (spdinv.hip)
constexpr int GJ_NB = 64;
hipError_t launch_gj_panel(const double *B, long ldb, Dim r, int b, double *D, double *Rrow, double *Ccol,
                           int *status, hipStream_t s);
hipError_t launch_gj_update(double *B, long ldb, Dim r, int b, const double *D, const double *Rrow,
                            const double *Ccol, hipStream_t s);

// operand slicing and sliced GEMM (ozaki.hip)
hipError_t launch_col_exponents(const double *X, long ldx, int rows, int cols, int *e, hipStream_t s);
hipError_t launch_row_exponents(const double *X, long ldx, int rows, int cols, int *e, hipStream_t s);
hipError_t launch_slice_cols(const double *X, long ldx, int rows, int cols, const int *e, int nslices,
                             __bf16 *planes, long ldp, long sp, hipStream_t s);
hipError_t launch_slice_rows_t(const double *X, long ldx, int rows, int cols, const int *e, int nslices,
                               __bf16 *planes, long ldp, long sp, hipStream_t s);
hipError_t launch_sliced_gemm(const SlicedGemmArgs &a, hipStream_t s);
long sliced_tiles(int M, int N, int lower);   // workgroups of one sliced-GEMM split
// weight classes of the chain's truncated pair set (t + u <= S)
constexpr int sliced_chain_classes(int S) { return S + 1 < 2 * S - 1 ? S + 1 : 2 * S - 1; }

// int8 modular product engine (modular.hip)
constexpr int MOD_MAX = 16;     // moduli (their product must fit 128 bits)
struct ModConsts {
    int n;                      // number of moduli
    int p[MOD_MAX];             // the moduli, pairwise coprime, <= 255
    int y[MOD_MAX];             // (M / p_l)^-1 mod p_l
    double pf[MOD_MAX], invp[MOD_MAX];
    double w1[MOD_MAX], w2[MOD_MAX], w3[MOD_MAX];   // M / p_l in three exact float64 pieces
    double m1, m2, m3;                              // M likewise
    double log2M;
};
struct ModGemmArgs {
    const int8_t *A; long lda; long sa;   // int8 residue plane l of opA at A + l sa: 1 KiB blocks of 16 rows x 64 k
    const int8_t *B; long ldb; long sb;   // (lda = ldb = Kpad bytes per row), see modular.hip
    int M, N, Kpad;                       // Kpad: multiple of 64, zero padded
    int lower;                            // tiles on or below the diagonal only (M == N)
    int cfg;                              // 0: 128 x 128 tiles, 1: 256 x 256 tiles
    int splitk;                           // K slices (each at most 1024 stages of 64)
    int8_t *R; long strideR;              // residues: plane (l, z) at R + (l splitk + z) strideR
    ModConsts mc;
};
struct ModRecArgs {
    const int8_t *R; long strideR;
    int M, N, lower, cfg, splitk, beta;
    const int *ea; const int *eb;         // row exponents of opA, column exponents of opB
    double *C; long ldc;
    ModConsts mc;
};
bool mod_consts(int N, ModConsts &mc);
int mod_beta(const ModConsts &mc, long K);
long mod_tiles(int M, int N, int lower, int cfg);     // workgroups of one modulus and K slice
int mod_min_splits(int Kpad);
size_t mod_residue_bytes(int M, int N, int lower, int cfg);   // bytes of one residue plane
hipError_t launch_mod_slice_cols(const double *X, long ldx, int rows, int cols, const int *e, int beta,
                                 const ModConsts &mc, int8_t *planes, long ldp, long sp, hipStream_t s);
hipError_t launch_mod_slice_rows_t(const double *X, long ldx, int rows, int cols, const int *e, int beta,
                                   const ModConsts &mc, int8_t *planes, long ldp, long sp, hipStream_t s);
hipError_t launch_mod_gemm(const ModGemmArgs &a, hipStream_t s);
hipError_t launch_mod_reconstruct(const ModRecArgs &a, hipStream_t s);

// incremental factorization (incremental.hip)
hipError_t launch_gather_rows(const double *X, long ldx, const int *idx, int r, int cols, double *out, long ldo,
                              hipStream_t s);
hipError_t launch_gather_cols_t(const double *X, long ldx, int row0, const int *idx, int r, int p, double *out,
                                long ldo, hipStream_t s);
hipError_t launch_offset_int(const int *src, int n, int off, int *dst, hipStream_t s);
hipError_t launch_trinv64(const double *T, long ldt, int r, double *Dinv, hipStream_t s);

// batched least squares (batched.hip)
constexpr int BATCH_NMAX = 256;
constexpr int BATCH_KMAX = 16;
hipError_t launch_batched(const void *desc, const int *order, int batch, int k, double tol, int nl, int *queue,
                          double *slabs, int grid, int nmax, int *rank, int *status, hipStream_t s);
hipError_t launch_batched_wide(const void *desc, const int *order, int batch, int k, double tol, int nl, int *queue,
                               double *slabs, int grid, int nmax, int *rank, int *status, hipStream_t s);
size_t batched_lds_bytes(int nl, int nmax, int k);
size_t batched_slab_doubles(int nmax, int k);
size_t batched_desc_bytes();
void batched_fill_desc(void *out, const float *G, const float *F, double *W, int m, int n, int ldg, int ldf, int ldw);
void batched_set_piv(void *desc, int b, int *piv);   // on a host copy of the descriptors

}  // namespace geninv
