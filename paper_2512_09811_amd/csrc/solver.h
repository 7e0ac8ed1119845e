// Frequency-window solver and the small dense FP64 kernels it uses.
#pragma once

#include "../../include/ppwin.h"
#include "context.h"

#include <exception>

namespace ppw {

struct SolveOptions {
  int precision = 0;      // 0 FP64 products, 1 FP32 products for the subspace
  double tol = 1e-9;
  int block = 0;
  int krylov_steps = 2;
  int max_basis = 480;
  int max_cycles = 200;
  double d_clamp = 1e-4;
  unsigned long long seed = 0;
  int correlated_f = 0;   // oscillator strengths from the property vector S mu (else mu)
  int method = 0;         // 0 folded inverse Krylov, 1 Riesz projector (contour filter)
  int contour_nodes = 6;  // Riesz: nodes on the upper half circle
  double contour_tol = 1e-4;  // Riesz: first-cycle solve tolerance (later: adaptive)
  int contour_maxit = 500;
  int pass_vectors = 0;   // most vectors per product pass (0: as the device budget allows)
};

// One window solve's request for A, B and S products of k orthonormal vectors V
// ([k][N] on the device, ready when 'ready' completes); the sink writes AV, BV, SV
// and records 'done' on the stream that wrote them.
struct ProductRequest {
  int id = 0;
  int k = 0;
  int prec = 0;  // 0: FP64 products, 1: FP32 contractions
  Context* ctx = nullptr;
  const double* V = nullptr;
  double *AV = nullptr, *BV = nullptr, *SV = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
  bool served = false;
  std::exception_ptr err;
};

// Where window solves send their product requests (blocking until served).
class ProductSink {
 public:
  virtual ~ProductSink() = default;
  virtual void multiply(ProductRequest& r) = 0;
};

// Largest number of vectors one window solve puts into a single product request.
int window_block_vectors(long N, int n_roots, const SolveOptions& opt);
// Device bytes one window solve allocates from its context's arena.
size_t window_solve_bytes(long N, int n_roots, const SolveOptions& opt);

// One window solve whose products go through 'sink' (shared with other solves).
// The context's product workspace must already hold window_block_vectors vectors.
void window_solve_shared(Context& c, const SolveOptions& opt, double omega0, int n_roots, ProductSink& sink, int id,
                         double* energies, double* vectors, double* osc, pp_solve_info* info);

// Roots of M z = omega Sigma z nearest omega0 (positive branch).  Host outputs.
// Throws NotConverged after writing all outputs when max_cycles is reached.
void window_solve(Context& c, const SolveOptions& opt, double omega0, int n_roots, double* energies,
                  double* vectors, double* osc, pp_solve_info* info);

// Several windows of one system solved concurrently (one host thread and stream
// each); their products are merged into shared product passes (two fixed groups of
// windows alternate passes).  Outputs are laid
// out window-major: energies[w][n_roots], vectors[w][n_roots][2][N], osc[w][n_roots],
// info[w].  Throws the first non-convergence after writing every output.
void window_solve_many(Context& c, const SolveOptions& opt, int nw, const double* omega0, int n_roots,
                       double* energies, double* vectors, double* osc, pp_solve_info* info);

// One-workgroup FP64 kernels on small n x n row-major matrices (n <= 512).
//  small_syev: A symmetric -> w ascending, Z[r*n + c] = component r of vector c.
//  scratch: 2 n^2 doubles (null: allocated and freed internally).
void small_syev(int n, const double* A, double* w, double* Z, hipStream_t s, double* scratch = nullptr);
//  small_cholesky: lower factor L (zeros above the diagonal); *info (device int,
//  may be null) = 0 on success, j+1 if the leading minor j is not positive.
void small_cholesky(int n, const double* A, double* L, int* info, hipStream_t s);
//  small_trinv: X = L^-1 for lower-triangular L.
void small_trinv(int n, const double* L, double* X, hipStream_t s);

}  // namespace ppw

namespace ppw {
// Partial symmetric eigensolver for the projected problem: the p eigenpairs of the
// n x n symmetric A (row-major, device) whose eigenvalues are nearest 'target'
// (p <= n, p <= 64).  lam[p] ascending; Z[n][p] row-major (column j = vector j).
// Work: 2 n^2 + 8 n p + 4 p^2 + 64 doubles of scratch (device).
// Returns q <= p, the number of independent pairs found (columns 0..q-1 valid).
int partial_syev(int n, const double* A, double target, int p, double* lam, double* Z, double* scratch,
                 hipStream_t s);
size_t partial_syev_scratch(int n, int p);
// Solve L^T X = B for lower-triangular L (n x n) and p right-hand sides B[n][p] (row-major, in place).
void small_trsm_lt(int n, const double* L, int p, double* B, hipStream_t s);
}  // namespace ppw
