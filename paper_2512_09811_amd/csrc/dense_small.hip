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
#include <algorithm>
#include <cfloat>
#include <vector>

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
// NT threads (1024 for the large projected problems; one wave for n <= 64, where the
// block-wide barriers of the rotation sweeps cost more than the arithmetic).  INLDS
// (n <= 64): W and Zr live in LDS instead of the scratch arrays passed in, so the
// sweeps run at LDS latency rather than at that of an L2 shared with concurrent GEMMs.
template <int NT, bool INLDS>
__global__ __launch_bounds__(NT) void syev_kernel(int n, const double* __restrict__ A, double* __restrict__ w,
                                                  double* __restrict__ Z, double* __restrict__ W,
                                                  double* __restrict__ Zr) {
  __shared__ double lds_w[INLDS ? 64 * 64 : 1], lds_z[INLDS ? 64 * 64 : 1];
  if (INLDS) {
    W = lds_w;
    Zr = lds_z;
  }
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
  for (long i = tid; i < nn; i += NT) W[i] = A[i];
  __syncthreads();

  // ---- Householder tridiagonalization (W <- H W H, u_k stored in column k) ----
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the reflected part (rows k+1..n-1)
    double part = 0.0;
    for (int r = tid; r < m; r += NT) {
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
      for (int r = tid; r < m; r += NT) u[r] = 0.0;
      __syncthreads();
      for (int r = tid; r < m; r += NT) W[(long)(k + 1 + r) * n + k] = 0.0;
      __syncthreads();
      continue;
    }
    const double alpha = x0 > 0 ? -xnorm : xnorm;
    // v = x - alpha e1, |v|^2 = 2 xnorm^2 - 2 x0 alpha
    const double vnorm = sqrt(2.0 * xx - 2.0 * x0 * alpha);
    for (int r = tid; r < m; r += NT) {
      const double x = W[(long)(k + 1 + r) * n + k];
      u[r] = (r == 0 ? x - alpha : x) / vnorm;
    }
    __syncthreads();
    // p = A22 u (column form, symmetric)
    for (int r = tid; r < m; r += NT) q[r] = 0.0;
    __syncthreads();
    for (int r = tid; r < m; r += NT) {
      double acc = 0.0;
      for (int cc = 0; cc < m; ++cc) acc += W[(long)(k + 1 + cc) * n + (k + 1 + r)] * u[cc];
      q[r] = acc;
    }
    __syncthreads();
    double kp = 0.0;
    for (int r = tid; r < m; r += NT) kp += u[r] * q[r];
    const double K = block_reduce_sum(kp, red);
    for (int r = tid; r < m; r += NT) q[r] = q[r] - K * u[r];
    __syncthreads();
    // A22 <- A22 - 2 (u q^T + q u^T)
    const long mm = (long)m * m;
    for (long idx = tid; idx < mm; idx += NT) {
      const int r = (int)(idx / m), cc = (int)(idx % m);
      W[(long)(k + 1 + r) * n + (k + 1 + cc)] -= 2.0 * (u[r] * q[cc] + q[r] * u[cc]);
    }
    if (tid == 0) {
      d[k] = W[(long)k * n + k];
      e[k] = alpha;
    }
    __syncthreads();
    for (int r = tid; r < m; r += NT) W[(long)(k + 1 + r) * n + k] = u[r];
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
  for (long i = tid; i < nn; i += NT) Zr[i] = ((i / n) == (i % n)) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    for (int r = tid; r < m; r += NT) u[r] = W[(long)(k + 1 + r) * n + k];
    __syncthreads();
    // t_c = sum_r u_r Z[k+1+r][k+1+c]
    for (int cc = tid; cc < m; cc += NT) {
      double acc = 0.0;
      for (int r = 0; r < m; ++r) acc += u[r] * Zr[(long)(k + 1 + r) * n + (k + 1 + cc)];
      q[cc] = acc;
    }
    __syncthreads();
    const long mm = (long)m * m;
    for (long idx = tid; idx < mm; idx += NT) {
      const int r = (int)(idx / m), cc = (int)(idx % m);
      Zr[(long)(k + 1 + r) * n + (k + 1 + cc)] -= 2.0 * u[r] * q[cc];
    }
    __syncthreads();
  }
  // column-major copy for the rotation phase: W[c*n + r] = Zr[r*n + c]
  for (long idx = tid; idx < nn; idx += NT) {
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
      const bool done = mm == l || ctl[2];
      // every thread holds its copy of ctl before thread 0 may rewrite it (for the
      // next sweep or the next l); without this barrier a late wave can read the
      // next values, miss the break and spin on a ctl that no thread updates
      __syncthreads();
      if (done) break;
      // apply rotations i = mm-1, mm-2, ... to columns (i, i+1) of Z, one row per thread
      for (int row = tid; row < n; row += NT) {
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
  for (int i = tid; i < n; i += NT) w[i] = d[perm[i]];
  for (long idx = tid; idx < nn; idx += NT) {
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

// Panel of the blocked Cholesky (one workgroup): columns j0..j0+jb-1 of the lower
// factor, in place in W (row-major n x n; only the lower triangle is read); the
// update of the trailing columns is a GEMM issued by the host.  info (nullable):
// 0 on success, j+1 for the first non-positive pivot j (later panels then stop).
__global__ __launch_bounds__(1024) void chol_panel_kernel(int n, int j0, int jb, double* __restrict__ W,
                                                         int* __restrict__ info) {
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) {
    if (info && j0 == 0) *info = 0;
    bad = (info && *info != 0) ? 1 : 0;
  }
  __syncthreads();
  if (bad) return;
  __shared__ double colj[64];  // column j of the panel rows j+1..kend-1 (jb <= 64)
  const int kend = j0 + jb;
  for (int j = j0; j < kend; ++j) {
    if (tid == 0) {
      const double d = W[(long)j * n + j];
      if (d > 0.0) {
        piv = sqrt(d);
        W[(long)j * n + j] = piv;
      } else {
        bad = 1;
        if (info) *info = j + 1;
      }
    }
    __syncthreads();
    if (bad) return;
    const double l = piv;
    for (int i = j + 1 + tid; i < n; i += blockDim.x) {
      const double x = W[(long)i * n + j] / l;
      W[(long)i * n + j] = x;
      if (i < kend) colj[i - j - 1] = x;
    }
    __syncthreads();
    // rest of the panel: W[i][k] -= W[i][j] W[k][j] for j < k < kend, k <= i; a wave
    // takes one row at a time (lane = column k), the waves interleave rows
    {
      const int lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
      const int k = j + 1 + lane;
      if (k < kend) {
        const double lkj = colj[lane];
        // eight rows per batch, all loads issued before the stores
        for (int i0 = j + 1 + wv; i0 < n; i0 += 8 * nw) {
          double a[8], b[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int i = i0 + nw * t;
            if (i < n) {
              a[t] = W[(long)i * n + j];
              b[t] = W[(long)i * n + k];
            }
          }
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int i = i0 + nw * t;
            if (i < n && k <= i) W[(long)i * n + k] = b[t] - a[t] * lkj;
          }
        }
      }
    }
    __syncthreads();
  }
}

__global__ void zero_upper_kernel(int n, double* __restrict__ L) {
  const long nn = (long)n * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < nn; idx += (long)gridDim.x * blockDim.x)
    if (idx % n > idx / n) L[idx] = 0.0;
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


// ---------------------------------------------------------------------------
// Spectrum slicing for the projected problem (only the eigenpairs near a target)
// ---------------------------------------------------------------------------

// Householder tridiagonalization (one workgroup).  d[n], e[n] (e[i] couples i, i+1);
// Hh[k][n] holds the unit reflector u_k of step k (zero in entries <= k).
//
// Step k reflects column k of the trailing block B (rows and columns k+1..n-1):
// u from that column, q = B u - (u.B u) u, then B -= 2 (u q^T + q u^T).  The kernel is
// bound by the bandwidth between the L2 and its one CU, so the rank-2 update of step k
// and the product B' u' of step k+1 share one sweep over the block: column k+1 of the
// updated block (which defines u') is formed first from the update formula, then every
// updated element of rows and columns k+2.. is written back and multiplied into B' u'
// in the same pass (one read and one write per element per step instead of two reads
// and one write).
__device__ __forceinline__ void reflector(int m, const double* __restrict__ col, double* __restrict__ u,
                                          double* red, double& alpha, bool& nonzero) {
  // u = (col - alpha e_0) / |col - alpha e_0| with alpha = -sign(col_0) |col|
  double part = 0.0;
  for (int r = threadIdx.x; r < m; r += blockDim.x) part += col[r] * col[r];
  const double xx = block_reduce_sum(part, red);
  const double x0 = col[0];
  const double xnorm = sqrt(xx);
  nonzero = xnorm != 0.0;
  alpha = x0 > 0 ? -xnorm : xnorm;
  if (!nonzero) return;
  const double vnorm = sqrt(2.0 * xx - 2.0 * x0 * alpha);
  for (int r = threadIdx.x; r < m; r += blockDim.x) u[r] = (r == 0 ? col[r] - alpha : col[r]) / vnorm;
  __syncthreads();
}

__global__ __launch_bounds__(kT) void tridiag_kernel(int n, const double* __restrict__ A, double* __restrict__ W,
                                                     double* __restrict__ dout, double* __restrict__ eout,
                                                     double* __restrict__ Hh) {
  __shared__ double u[kMaxN], q[kMaxN], un[kMaxN], qn[kMaxN], col[kMaxN];
  __shared__ double red[40];
  const int tid = threadIdx.x;
  const long nn = (long)n * n;
  for (long i = tid; i < nn; i += kT) {
    W[i] = A[i];
    Hh[i] = 0.0;
  }
  __syncthreads();
  // q = B u for the block of step k (rows/columns k+1..k+m), u in LDS
  auto symv = [&](int k, int m) {
    for (int r = tid; r < m; r += kT) {
      double acc = 0.0;
      for (int cc = 0; cc < m; ++cc) acc += W[(long)(k + 1 + cc) * n + (k + 1 + r)] * u[cc];
      q[r] = acc;
    }
    __syncthreads();
  };
  // reflector and product of step k from the stored column k (no pending update)
  bool refl = false;
  double alpha = 0.0;
  auto start_step = [&](int k) {
    const int m = n - k - 1;
    for (int r = tid; r < m; r += kT) col[r] = W[(long)(k + 1 + r) * n + k];
    __syncthreads();
    reflector(m, col, u, red, alpha, refl);
    if (refl) symv(k, m);
  };
  if (n >= 3) start_step(0);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    if (tid == 0) dout[k] = W[(long)k * n + k];
    if (!refl) {
      // column k is already reduced: nothing to apply
      if (tid == 0) eout[k] = 0.0;
      __syncthreads();
      if (k + 3 < n) start_step(k + 1);
      continue;
    }
    double kp = 0.0;
    for (int r = tid; r < m; r += kT) kp += u[r] * q[r];
    const double K = block_reduce_sum(kp, red);
    for (int r = tid; r < m; r += kT) {
      q[r] = q[r] - K * u[r];
      Hh[(long)k * n + k + 1 + r] = u[r];
    }
    if (tid == 0) eout[k] = alpha;
    __syncthreads();
    if (k + 3 < n) {
      // column k+1 of the updated block (rows k+2..) and its diagonal element
      for (int r = tid + 1; r < m; r += kT)
        col[r - 1] = W[(long)(k + 1 + r) * n + (k + 1)] - 2.0 * (u[r] * q[0] + q[r] * u[0]);
      if (tid == 0) W[(long)(k + 1) * n + (k + 1)] -= 2.0 * (u[0] * q[0] + q[0] * u[0]);
      __syncthreads();
      bool nref = false;
      double nalpha = 0.0;
      reflector(m - 1, col, un, red, nalpha, nref);
      // fused sweep over rows/columns k+2..n-1: update, and accumulate B' u'
      for (int c = tid + 1; c < m; c += kT) {
        const double qc = q[c], uc = u[c];
        double* Wc = W + (long)(k + 1) * n + (k + 1 + c);  // element (row r, this column) at Wc[r * n]
        double acc = 0.0;
        int r = 1;
        // twelve rows per batch: the loads are issued before any store of the batch, so
        // they are in flight together (a store to W could otherwise alias a later load)
        for (; r + 12 <= m; r += 12) {
          double w[12];
#pragma unroll
          for (int t = 0; t < 12; ++t) w[t] = Wc[(long)(r + t) * n];
#pragma unroll
          for (int t = 0; t < 12; ++t) {
            w[t] = w[t] - 2.0 * (u[r + t] * qc + q[r + t] * uc);
            Wc[(long)(r + t) * n] = w[t];
            if (nref) acc += w[t] * un[r + t - 1];
          }
        }
        for (; r < m; ++r) {
          const double w = Wc[(long)r * n] - 2.0 * (u[r] * qc + q[r] * uc);
          Wc[(long)r * n] = w;
          if (nref) acc += w * un[r - 1];
        }
        qn[c - 1] = acc;
      }
      __syncthreads();
      for (int r = tid; r < m - 1; r += kT) {
        u[r] = un[r];
        q[r] = qn[r];
      }
      refl = nref;
      alpha = nalpha;
      __syncthreads();
    } else {
      const long mm = (long)m * m;
      for (long idx = tid; idx < mm; idx += kT) {
        const int r = (int)(idx / m), cc = (int)(idx % m);
        W[(long)(k + 1 + r) * n + (k + 1 + cc)] -= 2.0 * (u[r] * q[cc] + q[r] * u[cc]);
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (n >= 2) {
      dout[n - 2] = W[(long)(n - 2) * n + (n - 2)];
      eout[n - 2] = W[(long)(n - 1) * n + (n - 2)];
    }
    dout[n - 1] = W[(long)(n - 1) * n + (n - 1)];
    eout[n - 1] = 0.0;
  }
}

// number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence)
__device__ int sturm_count(int n, const double* d, const double* e, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++c;
  }
  return c;
}

// Eigenvector of the tridiagonal (sd, se) for the eigenvalue lmb by inverse iteration:
// partially pivoted LU of T - lmb I (a zero pivot is replaced by pert), then four solves
// from a fixed start vector, each normalised.  The work arrays are private to the
// calling thread and do not overlap (restrict), so their loads can be issued ahead of
// the dependent recurrences.
__device__ void inverse_iteration(int n, const double* sd, const double* se, double lmb, double pert, int seed,
                                  double* __restrict__ dl, double* __restrict__ dd, double* __restrict__ du,
                                  double* __restrict__ du2, double* __restrict__ x, int* __restrict__ piv,
                                  double* __restrict__ out) {
  for (int i = 0; i < n; ++i) {
    dd[i] = sd[i] - lmb;
    if (i + 1 < n) {
      dl[i] = se[i];
      du[i] = se[i];
    }
    du2[i] = 0.0;
    piv[i] = i;
  }
  for (int i = 0; i + 1 < n; ++i) {
    if (fabs(dd[i]) >= fabs(dl[i])) {
      if (dd[i] == 0.0) dd[i] = pert;
      const double f = dl[i] / dd[i];
      dl[i] = f;
      dd[i + 1] -= f * du[i];
    } else {
      const double f = dd[i] / dl[i];
      dd[i] = dl[i];
      dl[i] = f;
      const double tmp = du[i];
      du[i] = dd[i + 1];
      dd[i + 1] = tmp - f * dd[i + 1];
      if (i + 2 < n) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
      piv[i] = i + 1;
    }
  }
  if (dd[n - 1] == 0.0) dd[n - 1] = pert;
  // deterministic start vector
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.5 * sin(0.7 * i + 1.3 * seed + 0.1);
  for (int iter = 0; iter < 4; ++iter) {
    double xi = x[0];
    for (int i = 0; i + 1 < n; ++i) {
      const double xn = x[i + 1];
      if (piv[i] == i) {
        x[i] = xi;
        xi = xn - dl[i] * xi;
      } else {
        x[i] = xn;
        xi = xi - dl[i] * xn;
      }
    }
    x[n - 1] = xi;
    double x1 = x[n - 1] / dd[n - 1];
    x[n - 1] = x1;
    double x2 = 0.0;
    if (n >= 2) {
      x2 = x1;
      x1 = (x[n - 2] - du[n - 2] * x2) / dd[n - 2];
      x[n - 2] = x1;
    }
    for (int i = n - 3; i >= 0; --i) {
      const double xi0 = (x[i] - du[i] * x1 - du2[i] * x2) / dd[i];
      x[i] = xi0;
      x2 = x1;
      x1 = xi0;
    }
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += x[i] * x[i];
    const double inv = 1.0 / sqrt(s2);
    for (int i = 0; i < n; ++i) x[i] *= inv;
  }
  for (int i = 0; i < n; ++i) out[i] = x[i];
}

// The p eigenvalues of the tridiagonal nearest 'target': the p below and the p above
// it by bisection (one per thread), the p nearest of those, then their vectors by
// inverse iteration with partially pivoted LU.  V[t][n]: vector t; lam[t] ascending;
// work: 6 n doubles per thread.  p <= 64.
__global__ __launch_bounds__(kT) void slice_kernel(int n, const double* __restrict__ d, const double* __restrict__ e,
                                                   double target, int p, double* __restrict__ lam,
                                                   double* __restrict__ V, double* __restrict__ work) {
  __shared__ double sd[kMaxN], se[kMaxN];
  __shared__ double bounds[3];
  __shared__ int lo_s, nc_s;
  __shared__ double cand[128];
  __shared__ int pick[64];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += kT) {
    sd[i] = d[i];
    se[i] = e[i];
  }
  __syncthreads();
  if (tid == 0) {
    double gl = sd[0], gu = sd[0], emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(se[i - 1]) : 0.0) + (i + 1 < n ? fabs(se[i]) : 0.0);
      gl = fmin(gl, sd[i] - r);
      gu = fmax(gu, sd[i] + r);
      if (i + 1 < n) emax = fmax(emax, se[i] * se[i]);
    }
    const double span = fmax(gu - gl, 1e-300);
    bounds[0] = gl - 1e-14 * span;
    bounds[1] = gu + 1e-14 * span;
    bounds[2] = fmax(DBL_MIN, 1e-300 + 4.0 * DBL_MIN * fmax(1.0, emax));
    // the p eigenvalues nearest the target lie among the p below and the p above it
    const int j0 = sturm_count(n, sd, se, target, bounds[2]);
    const int lo = max(0, j0 - p);
    lo_s = lo;
    nc_s = min(n, j0 + p) - lo;
  }
  __syncthreads();
  const double pivmin = bounds[2];
  const double scale = fmax(fabs(bounds[0]), fabs(bounds[1]));
  // bisection for every candidate index (ascending eigenvalue order)
  if (tid < nc_s) {
    const int idx = lo_s + tid;  // the idx-th smallest (0-based)
    double a = bounds[0], b = bounds[1];
    for (int it = 0; it < 200 && (b - a) > 4.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + DBL_MIN; ++it) {
      const double mid = 0.5 * (a + b);
      if (sturm_count(n, sd, se, mid, pivmin) > idx)
        b = mid;
      else
        a = mid;
    }
    cand[tid] = 0.5 * (a + b);
  }
  __syncthreads();
  // the p candidates nearest the target (ties: the lower), kept in ascending order;
  // candidates are ascending, so the nearest p form a contiguous run
  if (tid == 0) {
    int i0 = 0, i1 = nc_s;  // shrink [i0, i1) from the farther end
    while (i1 - i0 > p) {
      if (fabs(cand[i1 - 1] - target) >= fabs(cand[i0] - target))
        --i1;
      else
        ++i0;
    }
    for (int j = 0; j < p; ++j) pick[j] = i0 + j;
  }
  __syncthreads();
  if (tid < p) {
    const double lmb = cand[pick[tid]];
    lam[tid] = lmb;
    double* base = work + (long)tid * 6 * n;
    inverse_iteration(n, sd, se, lmb, 1e-15 * fmax(scale, 1e-300), tid, base, base + n, base + 2 * n, base + 3 * n,
                      base + 4 * n, (int*)(base + 5 * n), V + (long)tid * n);
  }
}

// T1[t][j] = UG[t][first + j] / sqrt(w[first + j])  (p x q, ld q)
__global__ void scale_keep_kernel(int p, int first, const double* __restrict__ U, const double* __restrict__ w,
                                  double* __restrict__ T1) {
  const int q = p - first;
  for (int idx = threadIdx.x; idx < p * q; idx += blockDim.x) {
    const int t = idx / q, j = idx % q;
    T1[idx] = U[(long)t * p + first + j] / sqrt(w[first + j]);
  }
}

__global__ void symmetrize_small_kernel(int n, double* A) {
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, c = idx % n;
    if (c > r) {
      const double m = 0.5 * (A[r * n + c] + A[c * n + r]);
      A[r * n + c] = m;
      A[c * n + r] = m;
    }
  }
}

// Y[t][i] = (T V)[t][i] for the tridiagonal (d, e) and p row vectors of length n
__global__ void tridiag_apply_kernel(int n, int p, const double* __restrict__ d, const double* __restrict__ e,
                                     const double* __restrict__ V, double* __restrict__ Y) {
  const long tot = (long)n * p;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot; idx += (long)gridDim.x * blockDim.x) {
    const int t = (int)(idx / n), i = (int)(idx % n);
    const double* v = V + (long)t * n;
    double y = d[i] * v[i];
    if (i > 0) y += e[i - 1] * v[i - 1];
    if (i + 1 < n) y += e[i] * v[i + 1];
    Y[idx] = y;
  }
}

// Z[r][j] = (H_0 ... H_{n-3} v_j)[r]: one workgroup per vector
__global__ __launch_bounds__(256) void backtransform_kernel(int n, int p, const double* __restrict__ Hh,
                                                            const double* __restrict__ V, double* __restrict__ Z) {
  __shared__ double v[kMaxN];
  __shared__ double red[40];
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += blockDim.x) v[i] = V[(long)j * n + i];
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const double* u = Hh + (long)k * n;
    double part = 0.0;
    for (int i = k + 1 + tid; i < n; i += blockDim.x) part += u[i] * v[i];
    // block reduction over 256 threads
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    const double dot = red[0] + red[1] + red[2] + red[3];
    for (int i = k + 1 + tid; i < n; i += blockDim.x) v[i] -= 2.0 * dot * u[i];
    __syncthreads();
  }
  for (int i = tid; i < n; i += blockDim.x) Z[(long)i * p + j] = v[i];
}

// L^T X = B, one workgroup per right-hand side (column j of B[n][p])
__global__ __launch_bounds__(256) void trsm_lt_kernel(int n, const double* __restrict__ L, int p, double* __restrict__ B) {
  __shared__ double b[kMaxN];
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += blockDim.x) b[i] = B[(long)i * p + j];
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const double xi = b[i] / L[(long)i * n + i];
    __syncthreads();
    if (tid == 0) b[i] = xi;
    // b[k] -= L[i][k] x_i for k < i   (row i of L, contiguous)
    for (int k = tid; k < i; k += blockDim.x) b[k] -= L[(long)i * n + k] * xi;
    __syncthreads();
  }
  for (int i = tid; i < n; i += blockDim.x) B[(long)i * p + j] = b[i];
}

}  // namespace

void small_syev(int n, const double* A, double* w, double* Z, hipStream_t s, double* scratch) {
  if (n < 1 || n > kMaxN) throw InvalidArg("small_syev: n out of range");
  double* ws = scratch;
  if (!ws) PPW_HIP(hipMalloc(&ws, sizeof(double) * 2 * (size_t)n * n));
  if (n <= 64)
    syev_kernel<64, true><<<1, 64, 0, s>>>(n, A, w, Z, ws, ws + (size_t)n * n);
  else
    syev_kernel<kT, false><<<1, kT, 0, s>>>(n, A, w, Z, ws, ws + (size_t)n * n);
  hipError_t e = hipGetLastError();
  if (!scratch) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(ws);
  }
  if (e != hipSuccess) throw DeviceError(std::string("syev launch: ") + hipGetErrorString(e));
}

size_t partial_syev_scratch(int n, int p) {
  return (size_t)2 * n * n + 2 * (size_t)n + 4 * (size_t)p * n + 6 * (size_t)n * p + 8 * (size_t)p * p + 64;
}

int partial_syev(int n, const double* A, double target, int p, double* lam, double* Z, double* scratch,
                 hipStream_t s) {
  if (n < 1 || n > kMaxN || p < 1 || p > 64 || p > n) throw InvalidArg("partial_syev: size out of range");
  double* W = scratch;
  double* Hh = W + (size_t)n * n;
  double* d = Hh + (size_t)n * n;
  double* e = d + n;
  double* V = e + n;
  double* V1 = V + (size_t)p * n;
  double* Y = V1 + (size_t)p * n;
  double* V2 = Y + (size_t)p * n;
  double* work = V2 + (size_t)p * n;
  double* G = work + (size_t)6 * n * p;
  double* UG = G + (size_t)p * p;
  double* T1 = UG + (size_t)p * p;
  double* H = T1 + (size_t)p * p;
  double* UH = H + (size_t)p * p;
  double* wG = UH + (size_t)p * p;
  double* eig_scr = wG + p;  // 2 p^2
  tridiag_kernel<<<1, kT, 0, s>>>(n, A, W, d, e, Hh);
  PPW_LAUNCH_CHECK();
  slice_kernel<<<1, kT, 0, s>>>(n, d, e, target, p, lam, V, work);
  PPW_LAUNCH_CHECK();
  // Rayleigh-Ritz inside span(V): G = V V^T, symmetric orthonormalization, H = V1 T V1^T
  GemmDesc g;
  g.M = p; g.N = p; g.K = n; g.transA = 0; g.lda = n; g.transB = 1; g.ldb = n; g.ldc = p;
  gemm_f64(g, 1.0, V, V, 0.0, G, s);
  small_syev(p, G, wG, UG, s, eig_scr);
  std::vector<double> wg(p);
  PPW_HIP(hipMemcpyAsync(wg.data(), wG, sizeof(double) * p, hipMemcpyDeviceToHost, s));
  PPW_HIP(hipStreamSynchronize(s));
  int first = 0;
  while (first < p && !(wg[first] > 1e-12 * wg[p - 1])) ++first;
  const int q = p - first;
  if (q == 0) throw Unstable("partial_syev: inverse iteration produced no independent vectors");
  scale_keep_kernel<<<1, 256, 0, s>>>(p, first, UG, wG, T1);
  PPW_LAUNCH_CHECK();
  // V1[j][r] = sum_t T1[t][j] V[t][r]   (T1 is p x q, ld q)
  GemmDesc a;
  a.M = q; a.N = n; a.K = p; a.transA = 1; a.lda = q; a.transB = 0; a.ldb = n; a.ldc = n;
  gemm_f64(a, 1.0, T1, V, 0.0, V1, s);
  tridiag_apply_kernel<<<(n * q + 255) / 256, 256, 0, s>>>(n, q, d, e, V1, Y);
  PPW_LAUNCH_CHECK();
  GemmDesc h;
  h.M = q; h.N = q; h.K = n; h.transA = 0; h.lda = n; h.transB = 1; h.ldb = n; h.ldc = q;
  gemm_f64(h, 1.0, V1, Y, 0.0, H, s);
  symmetrize_small_kernel<<<1, 256, 0, s>>>(q, H);
  small_syev(q, H, lam, UH, s, eig_scr);
  // V2[j][r] = sum_t UH[t][j] V1[t][r]
  GemmDesc b;
  b.M = q; b.N = n; b.K = q; b.transA = 1; b.lda = q; b.transB = 0; b.ldb = n; b.ldc = n;
  gemm_f64(b, 1.0, UH, V1, 0.0, V2, s);
  backtransform_kernel<<<q, 256, 0, s>>>(n, p, Hh, V2, Z);
  PPW_LAUNCH_CHECK();
  return q;
}

void small_trsm_lt(int n, const double* L, int p, double* B, hipStream_t s) {
  if (n < 1 || n > kMaxN) throw InvalidArg("small_trsm_lt: n out of range");
  trsm_lt_kernel<<<p, 256, 0, s>>>(n, L, p, B);
  PPW_LAUNCH_CHECK();
}

void small_cholesky(int n, const double* A, double* L, int* info, hipStream_t s) {
  if (n < 1 || n > kMaxN) throw InvalidArg("small_cholesky: n out of range");
  if (n <= 64) {
    cholesky_kernel<<<1, kT, 0, s>>>(n, A, L, info);
    PPW_LAUNCH_CHECK();
    return;
  }
  // blocked right-looking: panels of 64 columns in one workgroup, trailing updates as
  // GEMMs over the whole device (the unblocked sweep reads and writes the trailing
  // matrix once per column through one CU)
  constexpr int NB = 64;
  PPW_HIP(hipMemcpyAsync(L, A, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = std::min(NB, n - j0);
    chol_panel_kernel<<<1, 1024, 0, s>>>(n, j0, jb, L, info);
    PPW_LAUNCH_CHECK();
    const int j1 = j0 + jb, m2 = n - j1;
    if (m2 > 0) {
      GemmDesc d;
      d.M = m2;
      d.N = m2;
      d.K = jb;
      d.transA = 0;
      d.lda = n;
      d.transB = 1;
      d.ldb = n;
      d.ldc = n;
      const double* panel = L + (size_t)j1 * n + j0;
      gemm_f64(d, -1.0, panel, panel, 1.0, L + (size_t)j1 * n + j1, s);
    }
  }
  zero_upper_kernel<<<(n * n + 255) / 256, 256, 0, s>>>(n, L);
  PPW_LAUNCH_CHECK();
}

void small_trinv(int n, const double* L, double* X, hipStream_t s) {
  if (n < 1 || n > kMaxN) throw InvalidArg("small_trinv: n out of range");
  trinv_kernel<<<1, kT, 0, s>>>(n, L, X);
  PPW_LAUNCH_CHECK();
}

}  // namespace ppw
