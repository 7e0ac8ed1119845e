// One-workgroup FP64 dense kernels for the projected (subspace) problems.
//
// The subspace of the window solver never exceeds 512 vectors, so its symmetric
// eigenproblems, Cholesky factors and triangular inverses fit one workgroup: the
// matrices stay in global memory (L2-resident at these sizes), short vectors in
// LDS, and every parallel step is a row/column sweep by 1024 threads.
//
// Symmetric eigensolver: Householder reduction to tridiagonal form with explicit
// accumulation of the orthogonal factor, then the implicit QL iteration with
// Wilkinson-type shifts (the textbook tred2/tql2 pair), with the scalar
// recurrence run by one thread and each rotation sequence applied to all rows of
// the eigenvector matrix in parallel.  Eigenvalues are returned ascending.
#include <cfloat>

#include "solver.h"

namespace ppw {
namespace {

constexpr int kT = 1024;
constexpr int kMaxN = 512;

__device__ double block_reduce_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    red[32] = s;
  }
  __syncthreads();
  s = red[32];
  __syncthreads();
  return s;
}

// W: n x n working copy (row-major, symmetric), Zc: n x n, column-major eigenvectors.
__global__ __launch_bounds__(kT) void syev_kernel(int n, const double* __restrict__ A, double* __restrict__ w,
                                                  double* __restrict__ Z, double* __restrict__ W,
                                                  double* __restrict__ Zr) {
  __shared__ double u[kMaxN];
  __shared__ double q[kMaxN];
  __shared__ double d[kMaxN];
  __shared__ double e[kMaxN];
  __shared__ double cs[kMaxN];
  __shared__ double sn[kMaxN];
  __shared__ double red[40];
  __shared__ int ctl[4];
  const int tid = threadIdx.x;
  const long nn = (long)n * n;
  for (long i = tid; i < nn; i += kT) W[i] = A[i];
  __syncthreads();

  // ---- Householder tridiagonalization (W <- H W H, u_k stored in column k) ----
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the reflected part (rows k+1..n-1)
    double part = 0.0;
    for (int r = tid; r < m; r += kT) {
      const double x = W[(long)(k + 1 + r) * n + k];
      part += x * x;
    }
    const double xx = block_reduce_sum(part, red);
    const double x0 = W[(long)(k + 1) * n + k];
    const double xnorm = sqrt(xx);
    if (xnorm == 0.0) {
      if (tid == 0) {
        d[k] = W[(long)k * n + k];
        e[k] = 0.0;
      }
      for (int r = tid; r < m; r += kT) u[r] = 0.0;
      __syncthreads();
      for (int r = tid; r < m; r += kT) W[(long)(k + 1 + r) * n + k] = 0.0;
      __syncthreads();
      continue;
    }
    const double alpha = x0 > 0 ? -xnorm : xnorm;
    // v = x - alpha e1, |v|^2 = 2 xnorm^2 - 2 x0 alpha
    const double vnorm = sqrt(2.0 * xx - 2.0 * x0 * alpha);
    for (int r = tid; r < m; r += kT) {
      const double x = W[(long)(k + 1 + r) * n + k];
      u[r] = (r == 0 ? x - alpha : x) / vnorm;
    }
    __syncthreads();
    // p = A22 u (column form, symmetric)
    for (int r = tid; r < m; r += kT) q[r] = 0.0;
    __syncthreads();
    for (int r = tid; r < m; r += kT) {
      double acc = 0.0;
      for (int cc = 0; cc < m; ++cc) acc += W[(long)(k + 1 + cc) * n + (k + 1 + r)] * u[cc];
      q[r] = acc;
    }
    __syncthreads();
    double kp = 0.0;
    for (int r = tid; r < m; r += kT) kp += u[r] * q[r];
    const double K = block_reduce_sum(kp, red);
    for (int r = tid; r < m; r += kT) q[r] = q[r] - K * u[r];
    __syncthreads();
    // A22 <- A22 - 2 (u q^T + q u^T)
    const long mm = (long)m * m;
    for (long idx = tid; idx < mm; idx += kT) {
      const int r = (int)(idx / m), cc = (int)(idx % m);
      W[(long)(k + 1 + r) * n + (k + 1 + cc)] -= 2.0 * (u[r] * q[cc] + q[r] * u[cc]);
    }
    if (tid == 0) {
      d[k] = W[(long)k * n + k];
      e[k] = alpha;
    }
    __syncthreads();
    for (int r = tid; r < m; r += kT) W[(long)(k + 1 + r) * n + k] = u[r];
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = W[(long)(n - 2) * n + (n - 2)];
      e[n - 2] = W[(long)(n - 1) * n + (n - 2)];
    }
    d[n - 1] = W[(long)(n - 1) * n + (n - 1)];
    e[n - 1] = 0.0;
  }
  // ---- Q = H_0 H_1 ... H_{n-3}, accumulated backwards into Zr (row-major) ----
  for (long i = tid; i < nn; i += kT) Zr[i] = ((i / n) == (i % n)) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    for (int r = tid; r < m; r += kT) u[r] = W[(long)(k + 1 + r) * n + k];
    __syncthreads();
    // t_c = sum_r u_r Z[k+1+r][k+1+c]
    for (int cc = tid; cc < m; cc += kT) {
      double acc = 0.0;
      for (int r = 0; r < m; ++r) acc += u[r] * Zr[(long)(k + 1 + r) * n + (k + 1 + cc)];
      q[cc] = acc;
    }
    __syncthreads();
    const long mm = (long)m * m;
    for (long idx = tid; idx < mm; idx += kT) {
      const int r = (int)(idx / m), cc = (int)(idx % m);
      Zr[(long)(k + 1 + r) * n + (k + 1 + cc)] -= 2.0 * u[r] * q[cc];
    }
    __syncthreads();
  }
  // column-major copy for the rotation phase: W[c*n + r] = Zr[r*n + c]
  for (long idx = tid; idx < nn; idx += kT) {
    const long r = idx / n, cc = idx % n;
    W[cc * n + r] = Zr[idx];
  }
  __syncthreads();
  double* Zc = W;

  // ---- implicit QL on (d, e) ----
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      if (tid == 0) {
        int mm = l;
        for (; mm < n - 1; ++mm) {
          const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
          if (fabs(e[mm]) <= DBL_EPSILON * dd) break;
        }
        ctl[0] = mm;
        int nrot = 0;
        if (mm != l && iter < 100) {
          double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
          double r = hypot(g, 1.0);
          g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
          double s = 1.0, c = 1.0, p = 0.0;
          int i = mm - 1;
          bool early = false;
          for (; i >= l; --i) {
            const double f = s * e[i];
            const double b = c * e[i];
            r = hypot(f, g);
            e[i + 1] = r;
            if (r == 0.0) {
              d[i + 1] -= p;
              e[mm] = 0.0;
              early = true;
              break;
            }
            s = f / r;
            c = g / r;
            g = d[i + 1] - p;
            r = (d[i] - g) * s + 2.0 * c * b;
            p = s * r;
            d[i + 1] = g + p;
            g = c * r - b;
            cs[nrot] = c;
            sn[nrot] = s;
            ++nrot;
          }
          if (!early) {
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
          }
        }
        ctl[1] = nrot;
        ctl[2] = (mm != l && iter >= 100) ? 1 : 0;
      }
      __syncthreads();
      const int mm = ctl[0], nrot = ctl[1];
      if (mm == l || ctl[2]) break;
      // apply rotations i = mm-1, mm-2, ... to columns (i, i+1) of Z, one row per thread
      for (int row = tid; row < n; row += kT) {
        for (int t = 0; t < nrot; ++t) {
          const int i = mm - 1 - t;
          const double c = cs[t], s = sn[t];
          double* zi = Zc + (long)i * n + row;
          double* zj = Zc + (long)(i + 1) * n + row;
          const double f = *zj;
          *zj = s * (*zi) + c * f;
          *zi = c * (*zi) - s * f;
        }
      }
      __syncthreads();
      ++iter;
    }
  }
  __syncthreads();
  // ---- sort ascending (selection order by one thread), write outputs ----
  __shared__ int perm[kMaxN];
  if (tid == 0) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = 0; i < n; ++i) {
      int best = i;
      for (int j = i + 1; j < n; ++j)
        if (d[perm[j]] < d[perm[best]]) best = j;
      const int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kT) w[i] = d[perm[i]];
  for (long idx = tid; idx < nn; idx += kT) {
    const long r = idx / n, cc = idx % n;
    Z[idx] = Zc[(long)perm[cc] * n + r];
  }
}

__global__ __launch_bounds__(kT) void cholesky_kernel(int n, const double* __restrict__ A, double* __restrict__ L,
                                                      int* __restrict__ info) {
  __shared__ int bad;
  const int tid = threadIdx.x;
  const long nn = (long)n * n;
  for (long i = tid; i < nn; i += kT) {
    const long r = i / n, c = i % n;
    L[i] = c <= r ? A[i] : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double djj = L[(long)j * n + j];
    if (!(djj > 0.0)) {
      if (tid == 0) bad = j + 1;
      __syncthreads();
      break;
    }
    const double ljj = sqrt(djj);
    __syncthreads();
    if (tid == 0) L[(long)j * n + j] = ljj;
    for (int i = j + 1 + tid; i < n; i += kT) L[(long)i * n + j] /= ljj;
    __syncthreads();
    // trailing update of the lower triangle: L[i][k] -= L[i][j] L[k][j], j < k <= i
    const int m = n - j - 1;
    const long cnt = (long)m * m;
    for (long idx = tid; idx < cnt; idx += kT) {
      const int i = j + 1 + (int)(idx / m), k = j + 1 + (int)(idx % m);
      if (k <= i) L[(long)i * n + k] -= L[(long)i * n + j] * L[(long)k * n + j];
    }
    __syncthreads();
  }
  if (tid == 0 && info) *info = bad;
}

__global__ __launch_bounds__(kT) void trinv_kernel(int n, const double* __restrict__ L, double* __restrict__ X) {
  // thread j solves L x = e_j by forward substitution, column j of X
  for (int j = threadIdx.x; j < n; j += kT) {
    for (int i = 0; i < j; ++i) X[(long)i * n + j] = 0.0;
    for (int i = j; i < n; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) acc -= L[(long)i * n + k] * X[(long)k * n + j];
      X[(long)i * n + j] = acc / L[(long)i * n + i];
    }
  }
}

}  // namespace

void small_syev(int n, const double* A, double* w, double* Z, hipStream_t s, double* scratch) {
  if (n < 1 || n > kMaxN) throw InvalidArg("small_syev: n out of range");
  double* ws = scratch;
  if (!ws) PPW_HIP(hipMalloc(&ws, sizeof(double) * 2 * (size_t)n * n));
  syev_kernel<<<1, kT, 0, s>>>(n, A, w, Z, ws, ws + (size_t)n * n);
  hipError_t e = hipGetLastError();
  if (!scratch) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(ws);
  }
  if (e != hipSuccess) throw DeviceError(std::string("syev launch: ") + hipGetErrorString(e));
}

void small_cholesky(int n, const double* A, double* L, int* info, hipStream_t s) {
  if (n < 1 || n > kMaxN) throw InvalidArg("small_cholesky: n out of range");
  cholesky_kernel<<<1, kT, 0, s>>>(n, A, L, info);
  PPW_LAUNCH_CHECK();
}

void small_trinv(int n, const double* L, double* X, hipStream_t s) {
  if (n < 1 || n > kMaxN) throw InvalidArg("small_trinv: n out of range");
  trinv_kernel<<<1, kT, 0, s>>>(n, L, X);
  PPW_LAUNCH_CHECK();
}

}  // namespace ppw
