// Riesz projector of the pencil M z = omega Sigma z on a circular contour, applied to
// blocks of particle-hole vectors with the library's own products.
#pragma once

#include "context.h"

#include <functional>
#include <vector>

namespace ppw {

// A, B, S products of k vectors X ([k][N], device) into AV, BV, SV ([k][N], device),
// ordered on the caller's stream.
using ProductFn = std::function<void(int k, const double* X, double* AV, double* BV, double* SV)>;

struct ContourParams {
  double center = 0.0;  // circle center on the real axis (Ha)
  double radius = 0.0;  // circle radius (Ha)
  int nodes = 6;        // quadrature nodes on the upper half circle (2 * nodes in all)
  double tol = 1e-5;    // relative residual at which a shifted solve stops
  int maxit = 200;      // iteration cap of a shifted solve
};

// P = (1 / 2 pi i) closed-integral (z Sigma - M)^-1 Sigma dz by the trapezoidal rule on
// the circle: P v = (1/n) sum_{k<n} Re( r e^{i theta_k} x_k ), theta_k = pi (2k+1) / (2n),
// where x_k solves (z_k Sigma - M) x_k = Sigma v.  Every (node, vector) system is solved
// at once by conjugate-orthogonal CG (M and Sigma are real symmetric, so z Sigma - M is
// complex symmetric) preconditioned by its diagonal; one product pass per iteration
// serves all systems.
//
// Device layout: system s = node * k + column holds a complex 2N vector as four rows of
// N: real X, real Y, imaginary X, imaginary Y.
class ContourFilter {
 public:
  // kblock: largest number of 2N vectors per apply; nodes_max: largest node count;
  // chunk: largest product request (vectors) the product function accepts.
  ContourFilter(Context& c, int kblock, int nodes_max, int chunk, hipStream_t s);
  ~ContourFilter();
  ContourFilter(const ContourFilter&) = delete;
  ContourFilter& operator=(const ContourFilter&) = delete;

  // V: X rows [0, k) then Y rows [k, 2k) (device, [2k][N]); replaced by P applied to
  // each [X_j; Y_j].  Returns the largest iteration count of the shifted solves; the
  // largest final relative residual goes to *worst (if not null).
  int apply(const ContourParams& p, int k, double* V, const ProductFn& prod, double* worst = nullptr);

  // Device bytes the filter allocates (arena blocks rounded to 256 B).
  static size_t bytes(long N, int kblock, int nodes_max);
  long products() const { return products_; }

 private:
  Context& c_;
  hipStream_t s_;
  long N_;
  int kblock_, nodes_max_, chunk_;
  std::vector<void*> owned_;
  double *X_, *R_, *Z_, *P_, *Q_, *AP_, *BP_, *SP_;
  double *rho_, *rho2_, *sig_, *alpha_, *beta_, *rn2_, *bn2_, *zw_;
  int* done_;
  long products_ = 0;
  template <typename T>
  T* get(size_t n, const char* what);
  void multiply(int rows, const double* X, const ProductFn& prod);
};

}  // namespace ppw
