/*
 * Internal entry points of the ppwin library that the test-suite calls to check
 * single building blocks against plain references.  They are exported with the
 * ppint_ prefix, take device pointers, run synchronously on the default stream
 * and return a pp_status like the public API; hooks without a handle leave their error
 * message where pp_last_error(NULL) reads it.  They are not part of the stable
 * interface.
 */
#ifndef PPWIN_TESTING_H
#define PPWIN_TESTING_H

#include <stdint.h>

#include "ppwin.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C[b](m,n) = alpha * sum_kb sum_k A(m,k) B(k,n) + beta * C, the library GEMM
 * (layouts as in the library: transA = 0 -> A[m*lda+k], 1 -> A[k*lda+m]; transB = 0
 * -> B[k*ldb+n], 1 -> B[n*ldb+k]; batch b offsets b*sA, b*sB, b*sC; outer reduction
 * kb offsets kb*sAk, kb*sBk).  fp32 = 1 runs the FP32 matrix-core kernel on float
 * arrays, fp32 = 2 the split-BF16 kernel on float arrays (transA = 0, transB = 1, no
 * batch or outer reduction, else PP_EINVAL; the operands are copied into zero-padded
 * rows of a multiple of 8 values and split there, as the library does with its own),
 * fp32 = 3 the split-BF16 kernel on operands already in the split layout of
 * ppint_split_sbf16 (lda, ldb multiples of 8 and >= K, 16-byte aligned, else PP_EINVAL),
 * fp32 = 4 and 5 the same with its 128 x 128 or 256 x 256 tiles forced (for M, N >= 96).
 * ws_bytes of scratch are allocated for split-K (0 = no split). */
pp_status ppint_gemm(int32_t fp32, int32_t M, int32_t N, int32_t K, int32_t KB, int32_t nbatch, int32_t transA,
                     int64_t lda, int64_t sA, int64_t sAk, int32_t transB, int64_t ldb, int64_t sB, int64_t sBk,
                     int64_t ldc, int64_t sC, double alpha, const void* A, const void* B, double beta, void* C,
                     uint64_t ws_bytes);

/* ppint_gemm (fp32 as there) without batches or outer reduction, with C rows and columns split into
 * index pairs: C(m,n) = C[(m / cRm) * cSm + (m % cRm) * ldc + (n / cRn) * cSn + n % cRn]
 * (cRm = 0: m * ldc; cRn = 0: n).  Errors: PP_EINVAL for a negative split or a
 * shape the kernel cannot address. */
pp_status ppint_gemm_cmap(int32_t fp32, int32_t M, int32_t N, int32_t K, int32_t transA, int64_t lda, int32_t transB,
                          int64_t ldb, int64_t ldc, int32_t cRm, int64_t cSm, int32_t cRn, int64_t cSn, double alpha,
                          const void* A, const void* B, double beta, void* C, uint64_t ws_bytes);

/* Failure injection from the host: from now on, the after_calls-th HIP runtime call the
 * library checks reports the HIP error 'code' in place of its own return value (the
 * call itself runs as usual), so the entry point that made it fails with PP_EDEVICE and
 * the message of that error; the hook then disarms.  after_calls = 0 disarms it.  No
 * kernel or device state is touched.  PP_EINVAL for after_calls < 0 or a zero code. */
pp_status ppint_inject_hip_error(int32_t after_calls, int32_t code);

/* The split layout of the split-BF16 products, in place on n float values (device, n a
 * multiple of 8, 16-byte aligned): every chunk of 8 values becomes 8 bf16 hi parts
 * hi = bf16(x) (round to nearest even) followed by 8 bf16 lo parts lo = bf16(x - hi).
 * PP_EINVAL for other n or alignment. */
pp_status ppint_split_sbf16(int64_t n, float* x);

/* One member of ppint_gemm_group (layouts as in ppint_gemm, no batch). */
typedef struct {
  int32_t M, N, K, transA, transB;
  int64_t lda, ldb, ldc;
  const void* A;
  const void* B;
  void* C;
  double alpha, beta;
} ppint_gemm_member;

/* n independent GEMMs issued together: members sharing a tile shape are merged
 * into grouped launches when together they fill the chip (the path the serving
 * loop's merged product passes take); returns, in *grouped_launches (nullable),
 * how many grouped launches were made. */
pp_status ppint_gemm_group(int32_t fp32, int32_t n, const ppint_gemm_member* members, int32_t* grouped_launches);

/* Symmetric eigen-decomposition of an n x n row-major matrix A (device, lda = n)
 * by the library's one-workgroup FP64 solver: w ascending, Z columns = vectors
 * (row-major n x n, Z[r*n + c] = component r of vector c). */
pp_status ppint_syev(int32_t n, const double* A, double* w, double* Z);

/* The p eigenpairs of the symmetric n x n A (device, row-major) whose eigenvalues
 * are nearest 'target', by the library's partial solver (tridiagonalization,
 * bisection, inverse iteration, Rayleigh-Ritz in their span): lam[p] ascending,
 * Z[n][p] row-major (column j = vector j).  *q = number of pairs found (<= p). */
pp_status ppint_partial_syev(int32_t n, const double* A, double target, int32_t p, double* lam, double* Z,
                             int32_t* q);

/* Lower Cholesky factor of an SPD n x n matrix (device, row-major), in L. */
pp_status ppint_cholesky(int32_t n, const double* A, double* L);

/* Products of k particle-hole vectors by A, B, S at the given order (device
 * pointers, [k][n_occ][n_vir] each; SV may be NULL). fp32 selects the FP32
 * matrix-core path. */
pp_status ppint_products(pp_handle* h, int32_t order, int32_t k, const double* V, double* AV, double* BV,
                         double* SV, int32_t fp32);

/* Riesz projector of the handle's pencil (section on the connection to the Riesz
 * projector) applied to m vectors: out_j = (1/n) sum_{k<n} Re( r e^{i theta_k} x_k ),
 * theta_k = pi (2k+1) / (2n), z_k = center + radius e^{i theta_k}, where x_k solves
 * (z_k Sigma - M) x_k = Sigma V_j by diagonal-preconditioned conjugate-orthogonal CG to a
 * relative residual tol (at most maxit iterations).  V, out: device [m][2][n_occ][n_vir]
 * (X then Y of each vector); 1 <= m <= 64, 1 <= nodes <= 32.  *iters (nullable): largest
 * iteration count; *worst (nullable): largest final relative residual.  PP_EINVAL for
 * bad sizes, radius <= 0 or tol outside (0, 1). */
pp_status ppint_riesz_filter(pp_handle* h, double center, double radius, int32_t nodes, double tol, int32_t maxit,
                             int32_t m, const double* V, double* out, int32_t* iters, double* worst);

#ifdef __cplusplus
}
#endif

#endif /* PPWIN_TESTING_H */
