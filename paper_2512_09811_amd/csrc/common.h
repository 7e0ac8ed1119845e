// Shared declarations of the ppwin HIP library (gfx950 / CDNA4 only).
#pragma once

#include <vector>

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace ppw {

// Error raised inside the library; converted to a pp_status at the C ABI.
struct DeviceError : std::runtime_error {
  explicit DeviceError(const std::string& m) : std::runtime_error(m) {}
};
struct InvalidArg : std::runtime_error {
  explicit InvalidArg(const std::string& m) : std::runtime_error(m) {}
};
struct OutOfBudget : std::runtime_error {
  explicit OutOfBudget(const std::string& m) : std::runtime_error(m) {}
};
struct NotConverged : std::runtime_error {
  explicit NotConverged(const std::string& m) : std::runtime_error(m) {}
};
struct Unstable : std::runtime_error {
  explicit Unstable(const std::string& m) : std::runtime_error(m) {}
};
struct NotSupported : std::runtime_error {
  explicit NotSupported(const std::string& m) : std::runtime_error(m) {}
};

// Test hook (ppint_inject_hip_error): while armed, the n-th HIP call checked by PPW_HIP
// reports an injected error code in place of its own return value (the call itself ran).
hipError_t injected_hip_error(hipError_t e);

#define PPW_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = ::ppw::injected_hip_error(call);                                     \
    if (e_ != hipSuccess)                                                                \
      throw ::ppw::DeviceError(std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define PPW_LAUNCH_CHECK() PPW_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Batched, strided GEMM with an outer reduction loop.
//
//   C[b1,b2](m, n) = alpha * sum_{kb < KB} sum_{k < K} A[b1,b2,kb](m, k) B[b1,b2,kb](k, n)
//                    + beta * C[b1,b2](m, n)
//
// A(m,k) = A[m*lda + k] (transA = 0) or A[k*lda + m] (transA = 1), offset by
// b1*sA1 + b2*sA2 + kb*sAk elements; likewise B(k,n) = B[k*ldb + n] (transB = 0)
// or B[n*ldb + k] (transB = 1).  C(m,n) = C[m*ldc + n] + b1*sC1 + b2*sC2.
// beta == 0 never reads C.  The outer loop lets a contraction index that is
// split across two strides (e.g. (j, P) with P between j and the inner index)
// be reduced without a transpose.
//
// Rows and columns of C may each be pairs of indices with their own strides:
// with cRm > 0 row m is placed at (m / cRm) * cSm + (m % cRm) * ldc, with cRn > 0
// column n at (n / cRn) * cSn + n % cRn (0 leaves them plain), so a product whose
// output is a strided block of a larger array is written in place.  With a column
// split, column n is mapped as column cBn + n (a launch covering part of the columns).
// The strides cSm, cSn and the base cBn are non-negative.
//
// splitk > 0 fixes the number of reduction splits (1: none; the workspace must hold
// splitk * M * N * batches elements); 0 lets the launch choose.  tile = 64 selects the
// 64 x 64 tiles whatever the shape; 0 chooses by shape.
// ---------------------------------------------------------------------------
struct GemmDesc {
  int M = 0, N = 0, K = 0, KB = 1;
  int nb1 = 1, nb2 = 1;
  int transA = 0, transB = 0;
  long lda = 0, ldb = 0, ldc = 0;
  long sA1 = 0, sA2 = 0, sAk = 0;
  long sB1 = 0, sB2 = 0, sBk = 0;
  long sC1 = 0, sC2 = 0;
  int cRm = 0, cRn = 0, cBn = 0;
  long cSm = 0, cSn = 0;
  int splitk = 0, tile = 0;
};

// Workspace used by split-K launches (owned by the caller, bytes).
struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

void gemm_f64(const GemmDesc& d, double alpha, const double* A, const double* B, double beta,
              double* C, hipStream_t s, Workspace ws = {});
void gemm_f32(const GemmDesc& d, float alpha, const float* A, const float* B, float beta, float* C,
              hipStream_t s, Workspace ws = {});

// Same kernels under a separate symbol, used for the amplitude contraction H = tau G.
void gemm_f64_hhat(const GemmDesc& d, double alpha, const double* A, const double* B, double beta, double* C,
                   hipStream_t s, Workspace ws = {});
// Split-BF16 product (three BF16 MFMAs per FP32 product, FP32 accumulation, relative
// error about 2^-16) on operands held in the split layout of split_sbf16: operands
// contiguous along k with leading dimensions a multiple of 8 values (and >= K), 16-byte
// aligned, zero past K in a row's last chunk; no batch or outer reduction; C index splits
// allowed; d.tile = 128 or 256 fixes the tile shape (results do not depend on it).  Used
// for the amplitude contraction (and the amplitude strips' integrals) in PP_SPLIT_BF16 mode.
// amplitude = true launches the same kernel under the amplitude contraction's own symbol.
void gemm_sbf16(const GemmDesc& d, float alpha, const float* A, const float* B, float beta, float* C, hipStream_t s,
                bool amplitude = false);
// Splits n FP32 values in place (n a multiple of 8, x 16-byte aligned): each chunk of 8
// values becomes their 8 bf16 hi parts, hi = bf16(x) rounded to nearest even, followed
// by their 8 lo parts, lo = bf16(x - hi).
void split_sbf16(long n, float* x, hipStream_t s);
void gemm_f32_hhat(const GemmDesc& d, float alpha, const float* A, const float* B, float beta, float* C,
                   hipStream_t s, Workspace ws = {});

// Number of reduction splits a GEMM launch of d chooses by itself with a workspace of
// ws_bytes (FP64 or FP32 elements), so that an equivalent product laid out differently
// can be given the same splits (splitk) and round identically.
int gemm_auto_splitk(const GemmDesc& d, size_t ws_bytes, bool fp32);

// Algorithmic flop count of a GemmDesc (2 per multiply-add).
// One GEMM of a set issued together (C = alpha op(A) op(B) + beta C); tag 1 selects the
// kernel symbol of the amplitude contraction, tag 2 the split-BF16 kernel (operands in
// the split layout) and tag 3 that kernel under the amplitude contraction's symbol.  ws is the member's split-K workspace
// for when it is launched on its own.
template <typename T>
struct GemmCall {
  GemmDesc d;
  T alpha = T(1), beta = T(0);
  const T* A = nullptr;
  const T* B = nullptr;
  T* C = nullptr;
  Workspace ws;
  int tag = 0;
};

// Independent GEMMs (no member reads what another writes) on one stream, merged into
// grouped launches by tile shape.  Returns the number of grouped launches made.
int gemm_group_f64(const std::vector<GemmCall<double>>& calls, hipStream_t s);
int gemm_group_f32(const std::vector<GemmCall<float>>& calls, hipStream_t s);

inline double gemm_flops(const GemmDesc& d) {
  return 2.0 * d.M * (double)d.N * d.K * d.KB * d.nb1 * d.nb2;
}

}  // namespace ppw
