// Frequency-window solver: inverse Krylov basis from weighted-Jacobi steps,
// folded-spectrum selection, paired (X+Y, X-Y) Rayleigh-Ritz, residual refinement.
//
// Steps (subsection on interior eigenvalues of the Theory section):
//  * Z = M - omega0 Sigma; folded quotient rho(y) = |Z y|^2 / |y|^2.
//  * Inverse Krylov: each resolvent application (M - omega0 Sigma)^-1 v is replaced
//    by one weighted Jacobi sweep of Z x = v from x = v with the splitting Z = D + F:
//    direction d = D^-1 (v - Z v), new vector v + alpha d, alpha the stationary point
//    of the folded quotient (rho + a1 a + a2 a^2)/(1 + b1 a + b2 a^2) with the smaller
//    value (one product per step, since Z(v + a d) = Z v + a Z d).
//  * Every 2N vector [X; Y] contributes X and Y to an orthonormal basis Q of the
//    N-dimensional particle-hole space (classical Gram-Schmidt twice, then symmetric
//    orthonormalization that drops directions already in the span).  Products
//    (A+B)Q, (A-B)Q, SQ are computed for the orthonormal vectors themselves.
//  * The projected problem keeps the block structure of the pencil, so it is solved
//    exactly: Am = L L^T, K = L^T Sp^-1 Ap Sp^-1 L, K z = theta^2 z,
//    u = Sp^-1 L z / sqrt(theta), w = sqrt(theta) L^-T z  (u^T Sp w = 1).
//  * The window takes the n_roots positive Ritz pairs with the smallest folded
//    quotient at omega0; residuals r = (M - theta Sigma) y are computed in FP64 from
//    the stored products and turned into corrections by the diagonal of the shifted
//    pencil (2x2 solve per particle-hole pair in (u, w) coordinates).
//  * Thick restart keeps the X+Y and X-Y halves of the block's Ritz vectors.
// All arithmetic on vectors, projected matrices and small dense problems runs on the
// device in FP64; the host reads back only scalars per root (theta, residual norm,
// folded quotient) and eigenvalue lists that decide which directions to keep.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <exception>
#include <memory>
#include <mutex>
#include <thread>
#include <cmath>
#include <numeric>
#include <random>
#include <vector>

#include "kernels.h"
#include "riesz.h"
#include "solver.h"

namespace ppw {
namespace {

constexpr int kB = 256;
inline int gridn(long n) { return (int)std::max<long>(1, std::min<long>((n + kB - 1) / kB, 65536)); }

#define GS_LOOP(idx, n) for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (n); idx += (long)gridDim.x * blockDim.x)

__global__ void scale_rows_kernel(double* X, long N, int k, const double* __restrict__ s, int invert) {
  GS_LOOP(idx, N * k) {
    const int q = (int)(idx / N);
    X[idx] = invert ? X[idx] / s[q] : X[idx] * s[q];
  }
}

// coefficient matrices C[p][q] (ld): scale column q by s[q]
__global__ void scale_cols_kernel(double* C, int rows, int cols, long ld, const double* __restrict__ s, int mode) {
  GS_LOOP(idx, (long)rows * cols) {
    const int p = (int)(idx / cols), q = (int)(idx % cols);
    const double f = mode == 0 ? s[q] : (mode == 1 ? 1.0 / s[q] : (mode == 2 ? sqrt(s[q]) : 1.0 / sqrt(s[q])));
    C[(long)p * ld + q] *= f;
  }
}

__global__ void sqrt_kernel(double* x, int n) {
  GS_LOOP(i, n) x[i] = sqrt(x[i]);
}

__global__ void symmetrize_kernel(double* A, int n) {
  GS_LOOP(idx, (long)n * n) {
    const int r = (int)(idx / n), c = (int)(idx % n);
    if (c > r) {
      const double m = 0.5 * (A[(long)r * n + c] + A[(long)c * n + r]);
      A[(long)r * n + c] = m;
      A[(long)c * n + r] = m;
    }
  }
}

// T[j][jj] = U[j][keep[jj]] / sqrt(lam[keep[jj]]),  R[jj][j] = sqrt(lam[keep[jj]]) U[j][keep[jj]]
__global__ void symorth_factors_kernel(int kk, const double* __restrict__ U, const double* __restrict__ lam,
                                       const int* __restrict__ keep, int nk, double* __restrict__ T,
                                       double* __restrict__ R) {
  GS_LOOP(idx, (long)kk * nk) {
    const int j = (int)(idx / nk), jj = (int)(idx % nk);
    const int c = keep[jj];
    const double u = U[(long)j * kk + c];
    const double sl = sqrt(lam[c]);
    T[(long)j * nk + jj] = u / sl;
    R[(long)jj * kk + j] = sl * u;
  }
}

// Zt = 1/2 (PU + MW) - w0 SX,  Zb = 1/2 (PU - MW) + w0 SY
__global__ void zcombine_kernel(long n, double w0, const double* __restrict__ PU, const double* __restrict__ MW,
                                const double* __restrict__ SX, const double* __restrict__ SY, double* __restrict__ Zt,
                                double* __restrict__ Zb) {
  GS_LOOP(i, n) {
    const double a = 0.5 * (PU[i] + MW[i]), b = 0.5 * (PU[i] - MW[i]);
    Zt[i] = a - w0 * SX[i];
    Zb[i] = b + w0 * SY[i];
  }
}

__device__ __forceinline__ double clampd(double x, double c) {
  return fabs(x) < c ? (x >= 0 ? c : -c) : x;
}

// weighted-Jacobi direction: dX = (X - Zt)/clamp(dA - w0 dS), dY = (Y - Zb)/clamp(dA + w0 dS)
__global__ void jacobi_dir_kernel(long N, int k, double w0, double clampv, const double* __restrict__ dA,
                                  const double* __restrict__ dS, const double* __restrict__ X,
                                  const double* __restrict__ Y, const double* __restrict__ Zt,
                                  const double* __restrict__ Zb, double* __restrict__ dX, double* __restrict__ dY) {
  GS_LOOP(idx, N * k) {
    const long r = idx % N;
    dX[idx] = (X[idx] - Zt[idx]) / clampd(dA[r] - w0 * dS[r], clampv);
    dY[idx] = (Y[idx] - Zb[idx]) / clampd(dA[r] + w0 * dS[r], clampv);
  }
}

// alpha per column from the folded-quotient coefficients (see module comment)
__global__ void alpha_kernel(int k, const double* __restrict__ st, double* __restrict__ alpha) {
  // st layout: [6][k]: |Zt|^2+|Zb|^2 (rho nz^2), Z.Zd, |Zd|^2, c.cd, |cd|^2, |c|^2
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= k) return;
  const double nz2 = st[5 * k + q];
  const double rho = st[0 * k + q] / nz2;
  const double a1 = 2.0 * st[1 * k + q] / nz2;
  const double a2 = st[2 * k + q] / nz2;
  const double b1 = 2.0 * st[3 * k + q] / nz2;
  const double b2 = st[4 * k + q] / nz2;
  const double qa = a2 * b1 - a1 * b2, qb = 2.0 * (a2 - rho * b2), qc = a1 - rho * b1;
  double cand[2];
  int nc = 0;
  const double scale = fmax(fmax(fabs(qa), fabs(qb)), fmax(fabs(qc), 1e-300));
  if (fabs(qa) <= 1e-14 * scale) {
    if (qb != 0.0) cand[nc++] = -qc / qb;
  } else {
    const double disc = qb * qb - 4.0 * qa * qc;
    if (disc >= 0.0) {
      const double sq = sqrt(disc);
      const double qq = -0.5 * (qb + copysign(sq, qb));
      if (qq != 0.0) {
        cand[nc++] = qq / qa;
        cand[nc++] = qc / qq;
      } else {
        cand[nc++] = -qb / (2.0 * qa);
      }
    }
  }
  double best = 1.0, bestv = 0.0;
  bool have = false;
  for (int i = 0; i < nc; ++i) {
    const double x = cand[i];
    const double den = 1.0 + b1 * x + b2 * x * x;
    if (den <= 0.0) continue;
    const double val = (rho + a1 * x + a2 * x * x) / den;
    if (!have || val < bestv) {
      best = x;
      bestv = val;
      have = true;
    }
  }
  alpha[q] = best;
}

// C[:, q] += alpha[q] D[:, q] for coefficient matrices with ld
__global__ void axpy_cols_kernel(int rows, int k, long ld, const double* __restrict__ alpha, const double* __restrict__ D,
                                 long ldd, double* __restrict__ C) {
  GS_LOOP(idx, (long)rows * k) {
    const int p = (int)(idx / k), q = (int)(idx % k);
    C[(long)p * ld + q] += alpha[q] * D[(long)p * ldd + q];
  }
}

// Ritz residuals for every root j (vectors stored [j][N]):
//   ru = PU - th SW, rw = MW - th SU   (overwrite PU, MW);  fu = PU - w0 SW, fw = MW - w0 SU (norms only)
__global__ void residual_norms_kernel(long N, int nr, const double* __restrict__ th, double w0,
                                      double* __restrict__ PU, double* __restrict__ MW, const double* __restrict__ SU,
                                      const double* __restrict__ SW, double* __restrict__ out) {
  // one block per root; out[j] = |ru|^2 + |rw|^2, out[nr + j] = |fu|^2 + |fw|^2
  __shared__ double red[2][kB / 64];
  const int j = blockIdx.x;
  const long base = (long)j * N;
  const double t = th[j];
  double a = 0.0, b = 0.0;
  for (long i = threadIdx.x; i < N; i += blockDim.x) {
    const double pu = PU[base + i], mw = MW[base + i], su = SU[base + i], sw = SW[base + i];
    const double ru = pu - t * sw, rw = mw - t * su;
    const double fu = pu - w0 * sw, fw = mw - w0 * su;
    a += ru * ru + rw * rw;
    b += fu * fu + fw * fw;
    PU[base + i] = ru;
    MW[base + i] = rw;
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0, sb = 0;
    for (int w = 0; w < kB / 64; ++w) {
      sa += red[0][w];
      sb += red[1][w];
    }
    out[j] = sa;
    out[nr + j] = sb;
  }
}

// corrections for the listed roots: solve [[ap, -th s], [-th s, am]] [cu; cw] = -[ru; rw]
__global__ void correction_kernel(long N, int na, const int* __restrict__ idx_list, const double* __restrict__ th,
                                  double clampv, const double* __restrict__ dA, const double* __restrict__ dB,
                                  const double* __restrict__ dS, const double* __restrict__ RU,
                                  const double* __restrict__ RW, double* __restrict__ X, double* __restrict__ Y) {
  GS_LOOP(idx, N * na) {
    const int q = (int)(idx / N);
    const long r = idx % N;
    const int j = idx_list[q];
    const double t = th[j];
    const double ap = dA[r] + dB[r], am = dA[r] - dB[r], s = dS[r];
    const double det = clampd(ap * am - t * t * s * s, clampv);
    const double ru = RU[(long)j * N + r], rw = RW[(long)j * N + r];
    const double cu = -(am * ru + t * s * rw) / det;
    const double cw = -(t * s * ru + ap * rw) / det;
    X[idx] = 0.5 * (cu + cw);
    Y[idx] = 0.5 * (cu - cw);
  }
}

__global__ void gather_cols_kernel(int rows, int nsel, const int* __restrict__ sel, const double* __restrict__ src,
                                   long lds, double* __restrict__ dst, long ldd, int col0) {
  GS_LOOP(idx, (long)rows * nsel) {
    const int p = (int)(idx / nsel), q = (int)(idx % nsel);
    dst[(long)p * ldd + col0 + q] = src[(long)p * lds + sel[q]];
  }
}

__global__ void osc_kernel(int r, const double* __restrict__ T, const double* __restrict__ th, double* __restrict__ f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  double s = 0.0;
  for (int x = 0; x < 3; ++x) {
    const double t = sqrt(2.0) * T[(long)x * r + j];
    s += t * t;
  }
  f[j] = (2.0 / 3.0) * th[j] * s;
}

__global__ void pair_out_kernel(long N, int r, const double* __restrict__ U, const double* __restrict__ W,
                                double* __restrict__ out) {
  GS_LOOP(idx, 2 * N * r) {
    const long rr = idx % N;
    const long qh = idx / N;
    const int q = (int)(qh / 2), h = (int)(qh % 2);
    const double u = U[(long)q * N + rr], w = W[(long)q * N + rr];
    out[idx] = h == 0 ? 0.5 * (u + w) : 0.5 * (u - w);
  }
}

// start block: unit vectors on chosen pairs plus a small seeded perturbation (host-drawn)
__global__ void start_block_kernel(long N, int m, const int* __restrict__ pos, const double* __restrict__ noise,
                                   double* __restrict__ X, double* __restrict__ Y) {
  GS_LOOP(idx, N * m) {
    const int q = (int)(idx / N);
    const long r = idx % N;
    X[idx] = (r == pos[q] ? 1.0 : 0.0) + 1e-3 * noise[idx];
    Y[idx] = 1e-3 * noise[N * m + idx];
  }
}

// out[q] = A1[q].A2[q] + B1[q].B2[q] for vector sets [k][N] (one block per column)
__global__ void two_dots_kernel(const double* __restrict__ A1, const double* __restrict__ B1,
                                const double* __restrict__ A2, const double* __restrict__ B2, long N,
                                double* __restrict__ out) {
  __shared__ double red[kB / 64];
  const int q = blockIdx.x;
  const long base = (long)q * N;
  double a = 0.0;
  for (long i = threadIdx.x; i < N; i += blockDim.x) a += A1[base + i] * A2[base + i] + B1[base + i] * B2[base + i];
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kB / 64; ++w) s += red[w];
    out[q] = s;
  }
}

// out[q] = sum_p (X1[p][q] X2[p][q] + Y1[p][q] Y2[p][q]) over rows p < rows (ld)
__global__ void coeff_dots_kernel(int rows, int k, long ld, const double* __restrict__ X1,
                                  const double* __restrict__ Y1, const double* __restrict__ X2,
                                  const double* __restrict__ Y2, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= k) return;
  double s = 0.0;
  for (int p = 0; p < rows; ++p) s += X1[(long)p * ld + q] * X2[(long)p * ld + q] + Y1[(long)p * ld + q] * Y2[(long)p * ld + q];
  out[q] = s;
}

__global__ void identity_kernel(double* X, int n) {
  GS_LOOP(idx, (long)n * n) X[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
}

// out[0] = max |I - T| for an n x n matrix T
__global__ void ns_residual_kernel(int n, const double* __restrict__ T, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (long idx = threadIdx.x; idx < (long)n * n; idx += blockDim.x)
    m = fmax(m, fabs(T[idx] - ((idx / n == idx % n) ? 1.0 : 0.0)));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void copy_cols_kernel(int rows, int cols, const double* __restrict__ src, long lds, double* __restrict__ dst,
                                 long ldd) {
  GS_LOOP(idx, (long)rows * cols) {
    const int r = (int)(idx / cols), c = (int)(idx % cols);
    dst[(long)r * ldd + c] = src[(long)r * lds + c];
  }
}

// out[j] = sum_p (U[p][j]^2 + W[p][j]^2)
// X = (u + w) / 2, Y = (u - w) / 2 for paired halves u = X + Y, w = X - Y ([k][N] each)
__global__ void halves_kernel(long n, const double* __restrict__ U, const double* __restrict__ W,
                              double* __restrict__ X, double* __restrict__ Y) {
  GS_LOOP(i, n) {
    X[i] = 0.5 * (U[i] + W[i]);
    Y[i] = 0.5 * (U[i] - W[i]);
  }
}

__global__ void coeff_norms_kernel(int rows, int cols, const double* __restrict__ U, const double* __restrict__ W,
                                   double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int p = 0; p < rows; ++p) s += U[(long)p * cols + j] * U[(long)p * cols + j] + W[(long)p * cols + j] * W[(long)p * cols + j];
  out[j] = s;
}

GemmDesc gd(int M, int N, int K, int tA, long lda, int tB, long ldb, long ldc) {
  GemmDesc d;
  d.M = M;
  d.N = N;
  d.K = K;
  d.transA = tA;
  d.lda = lda;
  d.transB = tB;
  d.ldb = ldb;
  d.ldc = ldc;
  return d;
}

// ---------------------------------------------------------------------------
// Merges the product requests of concurrently running window solves of one system
// into a single product pass.  Each window thread submits its block (recorded as
// ready on its own stream) and blocks; when every active window has submitted, the
// last one runs the pass on the system's stream and the results are copied back,
// with a completion event per request.  Requests are served in window order, so the
// batch composition (and therefore every rounding) is a deterministic function of
// the inputs.
// Merges the product requests of a group of windows of one system into shared
// passes: a pass runs when every window of the group still solving has a request
// pending.  Several groups may share a context: 'enqueue' serializes their passes
// on the context's stream (and its product workspace).
class ProductBatcher : public ProductSink {
 public:
  using Req = ProductRequest;
  ProductBatcher(Context& c, int active, int precision, std::mutex* enqueue, int max_pass = 0)
      : c_(c), active_(active), prec_(precision), enqueue_(enqueue), max_pass_(max_pass) {}
  ~ProductBatcher() override {
    for (void* q : bufs_) c_.arena.free(q);
  }
  void reserve(int ktot) {
    const size_t n = (size_t)ktot * c_.N;
    V_ = c_.arena.alloc<double>(n, "batch V");
    AV_ = c_.arena.alloc<double>(n, "batch AV");
    BV_ = c_.arena.alloc<double>(n, "batch BV");
    SV_ = c_.arena.alloc<double>(n, "batch SV");
    bufs_ = {V_, AV_, BV_, SV_};
    cap_ = ktot;
    // vectors per product pass: all of them when their product workspaces fit the
    // device budget, else the largest count that fits (a batch then runs as several
    // passes; with amplitudes rebuilt in strips each pass rebuilds them)
    size_t avail;
    if (c_.arena.budget()) {
      avail = c_.arena.budget() > c_.arena.used() ? c_.arena.budget() - c_.arena.used() : 0;
    } else {
      size_t freeb = 0, total = 0;
      PPW_HIP(hipMemGetInfo(&freeb, &total));
      avail = (size_t)(0.9 * (double)freeb);
    }
    auto need = [&](int q) { return sigma_reserve_bytes(c_, q, 0) + (prec_ == 1 ? sigma_reserve_bytes(c_, q, 1) : 0); };
    chunk_ = max_pass_ > 0 ? std::min(ktot, max_pass_) : ktot;
    while (chunk_ > 1 && need(chunk_) > avail) --chunk_;
    sigma_reserve(c_, chunk_, 0);
    if (prec_ == 1) sigma_reserve(c_, chunk_, 1);
  }
  int chunk() const { return chunk_; }
  void multiply(Req& r) override {
    std::unique_lock<std::mutex> lk(mu_);
    r.served = false;
    pending_.push_back(&r);
    if ((int)pending_.size() >= active_)
      serve();
    else
      cv_.wait(lk, [&] { return r.served; });
    if (r.err) std::rethrow_exception(r.err);
  }
  void leave() {
    std::unique_lock<std::mutex> lk(mu_);
    --active_;
    if (active_ > 0 && (int)pending_.size() >= active_) serve();
  }

 private:
  void serve() {
    std::exception_ptr err;
    std::sort(pending_.begin(), pending_.end(), [](const Req* a, const Req* b) { return a->id < b->id; });
    std::unique_lock<std::mutex> eq(*enqueue_);
    try {
      hipStream_t s = c_.stream;
      const long N = c_.N;
      for (int prec = 0; prec < 2; ++prec) {
        int kt = 0;
        for (auto* r : pending_)
          if (r->prec == prec) kt += r->k;
        if (kt == 0) continue;
        if (kt > cap_) throw InvalidArg("product batch exceeds its reserved size");
        long off = 0;
        for (auto* r : pending_) {
          if (r->prec != prec) continue;
          PPW_HIP(hipStreamWaitEvent(s, r->ready, 0));
          PPW_HIP(hipMemcpyAsync(V_ + off * N, r->V, sizeof(double) * r->k * N, hipMemcpyDeviceToDevice, s));
          off += r->k;
        }
        // passes of equal size (each at most chunk_ vectors)
        const int npass = (kt + chunk_ - 1) / chunk_;
        const int per = (kt + npass - 1) / npass;
        for (int c0 = 0; c0 < kt; c0 += per) {
          const int kc = std::min(per, kt - c0);
          const size_t o0 = (size_t)c0 * N;
          if (prec == 1)
            sigma_core_f32(c_, c_.order, kc, V_ + o0, AV_ + o0, BV_ + o0, SV_ + o0);
          else
            sigma_core(c_, c_.order, kc, V_ + o0, AV_ + o0, BV_ + o0, SV_ + o0);
          if (trace_) {
            // progress of long passes (the wait serializes the passes; tracing only)
            PPW_HIP(hipStreamSynchronize(s));
            std::fprintf(stderr, "[ppwin] product pass of %d vectors (%s) done\n", kc, prec ? "reduced" : "FP64");
          }
        }
        off = 0;
        for (auto* r : pending_) {
          if (r->prec != prec) continue;
          const size_t b = sizeof(double) * r->k * N;
          PPW_HIP(hipMemcpyAsync(r->AV, AV_ + off * N, b, hipMemcpyDeviceToDevice, s));
          PPW_HIP(hipMemcpyAsync(r->BV, BV_ + off * N, b, hipMemcpyDeviceToDevice, s));
          PPW_HIP(hipMemcpyAsync(r->SV, SV_ + off * N, b, hipMemcpyDeviceToDevice, s));
          PPW_HIP(hipEventRecord(r->done, s));
          off += r->k;
        }
      }
    } catch (...) {
      err = std::current_exception();
    }
    for (auto* r : pending_) {
      r->err = err;
      r->served = true;
    }
    pending_.clear();
    cv_.notify_all();
  }
  Context& c_;
  int active_;
  int prec_;
  std::mutex* enqueue_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::vector<Req*> pending_;
  double *V_ = nullptr, *AV_ = nullptr, *BV_ = nullptr, *SV_ = nullptr;
  std::vector<void*> bufs_;
  int cap_ = 0;
  int chunk_ = 0;
  int max_pass_ = 0;
  bool trace_ = std::getenv("PPWIN_TRACE") != nullptr;
};

// Block size, basis limit and vectors per extension of one window solve (as the
// Solver constructor sets them).
struct SolverDims {
  int m, nbmax, kmax;
};
SolverDims solver_dims(long N, int nroots, const SolveOptions& o) {
  SolverDims d;
  // the Riesz subspace iteration needs more vectors than roots (the filter separates the
  // window from its neighbours through the block's extra vectors)
  d.m = o.block > 0 ? o.block : (o.method == 1 ? 2 * nroots : nroots + 2);
  d.m = (int)std::min<long>(d.m, N);
  d.nbmax = (int)std::min<long>(o.max_basis > 0 ? o.max_basis : 480, N);
  d.nbmax = std::max(d.nbmax, std::min<int>((int)N, 2 * d.m));
  d.kmax = 2 * d.m;
  return d;
}


class Solver {
 public:
  Solver(Context& c, const SolveOptions& o, double w0, int nroots, ProductSink* pb, int id)
      : c_(c), opt_(o), w0_(w0), nr_(nroots), N_(c.N), pb_(pb), id_(id) {
    const SolverDims dm = solver_dims(N_, nroots, o);
    m_ = dm.m;
    nbmax_ = dm.nbmax;
    kmax_ = dm.kmax;  // new vectors per extension (X and Y halves of a block)
    trace_ = std::getenv("PPWIN_TRACE") != nullptr;
    PPW_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    PPW_HIP(hipEventCreateWithFlags(&ev_ready_, hipEventDisableTiming));
    PPW_HIP(hipEventCreateWithFlags(&ev_done_, hipEventDisableTiming));
    alloc();
    if (opt_.method == 1) cf_.reset(new ContourFilter(c_, m_, opt_.contour_nodes, kmax_, s_));
  }
  ~Solver() {
    if (s_) (void)hipStreamSynchronize(s_);
    cf_.reset();
    for (void* p : owned_) c_.arena.free(p);
    if (ev_ready_) (void)hipEventDestroy(ev_ready_);
    if (ev_done_) (void)hipEventDestroy(ev_done_);
    if (s_) (void)hipStreamDestroy(s_);
  }
  int kmax() const { return kmax_; }

  void run(double* energies, double* vectors, double* osc, pp_solve_info* info);

 private:
  Context& c_;
  SolveOptions opt_;
  double w0_;
  int nr_, m_, nbmax_, kmax_;
  hipStream_t s_ = nullptr;
  long N_;
  ProductSink* pb_;
  int id_;
  hipEvent_t ev_ready_ = nullptr, ev_done_ = nullptr;
  bool trace_ = false;  // per-cycle progress on stderr when PPWIN_TRACE is set
  bool refined_ = false;  // mixed precision: every product FP64 from here on
  Workspace wsp_;
  int nb_ = 0;
  int rld_ = 1;  // columns (leading dimension) of the current Ritz coefficient matrices us_/ws_
  std::vector<void*> owned_;
  // basis and products [nbmax][N]
  double *Q_, *P0_, *P1_, *PS_, *Qs_, *P0s_, *P1s_, *PSs_;
  // work vectors [*][N]
  double *V_, *AV_, *BV_, *SV_, *T1_, *T2_, *T3_, *T4_, *T5_, *T6_;
  // Ritz-space arrays [nbmax][N]
  double *RU_, *RW_, *RSU_, *RSW_;
  // small matrices
  double *c1_, *c2_, *g_, *U_, *lam_, *Tm_, *Rm_, *Ctot_, *Rtot_, *tmp_, *tmp2_, *nrm_;
  double *cx_, *cy_, *cdx_, *cdy_, *cu_, *cw_, *st_, *alpha_;
  double *Ap_, *Am_, *Sp_, *L_, *Li_, *Ls_, *Lsi_, *Spi_, *K_, *th2_, *Zk_, *us_, *ws_, *th_, *stats_;
  double *eigscr_;
  int *keep_, *ival_, *sel_;
  double* noise_;
  long products_ = 0;
  // Riesz projector mode: contour filter, circle radius around omega0, solve iterations
  std::unique_ptr<ContourFilter> cf_;
  double rad_ = 0.0;
  long contour_iters_ = 0;
  double contour_worst_ = 1.0;  // worst residual of the window when the block was formed

  template <typename T>
  T* get(size_t n, const char* w) {
    const size_t bytes = ((n * sizeof(T) + 255) / 256) * 256;  // the arena's block rounding
    if (sizing_) {
      slab_need_ += bytes;
      return nullptr;
    }
    if (slab_ && slab_off_ + bytes <= slab_need_) {
      T* p = reinterpret_cast<T*>(slab_ + slab_off_);
      slab_off_ += bytes;
      return p;
    }
    T* p = c_.arena.alloc<T>(n, w);
    owned_.push_back(p);
    return p;
  }
  // The solver's buffers are carved from one arena block: a sizing pass adds up their
  // rounded sizes, then a single allocation (one hipMalloc instead of about seventy) is
  // cut in the same order.
  size_t slab_need_ = 0, slab_off_ = 0;
  char* slab_ = nullptr;
  bool sizing_ = false;
  void alloc() {
    sizing_ = true;
    carve();
    sizing_ = false;
    slab_ = c_.arena.alloc<char>(slab_need_, "window solver buffers");
    owned_.push_back(slab_);
    carve();
    PPW_HIP(hipMemsetAsync(Q_, 0, sizeof(double) * (size_t)nbmax_ * N_, s_));
  }
  void carve() {
    const size_t bN = (size_t)nbmax_ * N_;
    const size_t kN = (size_t)kmax_ * N_;
    Q_ = get<double>(bN, "basis Q");
    P0_ = get<double>(bN, "basis (A+B)Q");
    P1_ = get<double>(bN, "basis (A-B)Q");
    PS_ = get<double>(bN, "basis SQ");
    Qs_ = get<double>(bN, "basis swap");
    P0s_ = get<double>(bN, "basis swap");
    P1s_ = get<double>(bN, "basis swap");
    PSs_ = get<double>(bN, "basis swap");
    RU_ = get<double>(bN, "ritz PU");
    RW_ = get<double>(bN, "ritz MW");
    RSU_ = get<double>(bN, "ritz SU");
    RSW_ = get<double>(bN, "ritz SW");
    V_ = get<double>(kN, "block V");
    AV_ = get<double>(kN, "block AV");
    BV_ = get<double>(kN, "block BV");
    SV_ = get<double>(kN, "block SV");
    T1_ = get<double>(kN, "block tmp");
    T2_ = get<double>(kN, "block tmp");
    T3_ = get<double>(kN, "block tmp");
    T4_ = get<double>(kN, "block tmp");
    T5_ = get<double>(kN, "block tmp");
    T6_ = get<double>(kN, "block tmp");
    const size_t bk = (size_t)nbmax_ * kmax_;
    const size_t bb = (size_t)nbmax_ * nbmax_;
    const size_t kk = (size_t)kmax_ * kmax_;
    c1_ = get<double>(bk, "c1");
    c2_ = get<double>(bk, "c2");
    g_ = get<double>(std::max(kk, bb), "gram");
    U_ = get<double>(std::max(kk, bb), "eigvec");
    lam_ = get<double>(nbmax_, "eigval");
    Tm_ = get<double>(std::max(kk, bk), "T");
    Rm_ = get<double>(kk, "R");
    Ctot_ = get<double>(bk, "C");
    Rtot_ = get<double>(kk, "R tot");
    tmp_ = get<double>(std::max(bk, bb), "tmp");
    tmp2_ = get<double>(std::max(bk, bb), "tmp2");
    nrm_ = get<double>(std::max(kmax_, 8), "norms");
    cx_ = get<double>(bk, "cx");
    cy_ = get<double>(bk, "cy");
    cdx_ = get<double>(bk, "cdx");
    cdy_ = get<double>(bk, "cdy");
    cu_ = get<double>(bk, "cu");
    cw_ = get<double>(bk, "cw");
    st_ = get<double>((size_t)8 * kmax_, "stats");
    alpha_ = get<double>(kmax_, "alpha");
    Ap_ = get<double>(bb, "Ap");
    Am_ = get<double>(bb, "Am");
    Sp_ = get<double>(bb, "Sp");
    L_ = get<double>(bb, "L");
    Li_ = get<double>(bb, "Li");
    Ls_ = get<double>(bb, "Ls");
    Lsi_ = get<double>(bb, "Lsi");
    Spi_ = get<double>(bb, "Spi");
    K_ = get<double>(bb, "K");
    th2_ = get<double>(nbmax_, "theta2");
    Zk_ = get<double>(bb, "Zk");
    us_ = get<double>(bb, "us");
    ws_ = get<double>(bb, "ws");
    th_ = get<double>(nbmax_, "theta");
    stats_ = get<double>(std::max((size_t)2 * nbmax_, (size_t)3 * 64), "ritz stats");
    eigscr_ = get<double>(std::max((size_t)2 * std::max(bb, kk), partial_syev_scratch(nbmax_, 64)), "eig scratch");
    keep_ = get<int>(std::max(kmax_, nbmax_), "keep");
    ival_ = get<int>(4, "info");
    sel_ = get<int>(std::max(kmax_, nbmax_), "sel");
    noise_ = get<double>((size_t)2 * m_ * N_, "noise");
    wsp_.bytes = (size_t)32 << 20;
    wsp_.ptr = get<char>(wsp_.bytes, "solver split-K workspace");
  }

  void gemm(const GemmDesc& d, double a, const double* A, const double* B, double b, double* C) {
    gemm_f64(d, a, A, B, b, C, s_, wsp_);
  }
  template <typename T>
  std::vector<T> fetch(const T* p, size_t n) {
    std::vector<T> h(n);
    if (n) {
      PPW_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s_));
      PPW_HIP(hipStreamSynchronize(s_));
    }
    return h;
  }
  template <typename T>
  void upload(T* d, const std::vector<T>& h) {
    if (h.empty()) return;
    PPW_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s_));
  }
  // C[p][q] = sum_r X[p][r] Y[q][r] for row-major vector sets (ldc = ldc)
  void tn(int p, int q, const double* X, const double* Y, double* C, long ldc, double beta = 0.0) {
    gemm(gd(p, q, (int)N_, 0, N_, 1, N_, ldc), 1.0, X, Y, beta, C);
  }
  // Out[q][r] = alpha sum_p C[p][q] Basis[p][r] + beta Out
  void expand(int q, int p, const double* C, long ldc, const double* Basis, double* Out, double alpha = 1.0,
              double beta = 0.0) {
    if (p == 0) {
      if (beta == 0.0) PPW_HIP(hipMemsetAsync(Out, 0, sizeof(double) * q * N_, s_));
      return;
    }
    gemm(gd(q, (int)N_, p, 1, ldc, 0, N_, N_), alpha, C, Basis, beta, Out);
  }
  // small: C = A(m x k, lda) * B(k x n, ldb)
  void small_mm(int m, int n, int k, const double* A, long lda, int tA, const double* B, long ldb, int tB, double* C,
                long ldc, double alpha = 1.0, double beta = 0.0) {
    gemm(gd(m, n, k, tA, lda, tB, ldb, ldc), alpha, A, B, beta, C);
  }

  // A, B, S products of k orthonormal vectors X (device, [k][N]) into AV_, BV_, SV_,
  // merged with the other windows' requests by the batcher
  void products(int k, const double* X, bool exact) { products_into(k, X, AV_, BV_, SV_, exact); }
  void products_into(int k, const double* X, double* AV, double* BV, double* SV, bool exact) {
    ProductRequest r;
    r.id = id_;
    r.ctx = &c_;
    r.k = k;
    r.prec = (exact || opt_.precision != 1 || refined_) ? 0 : 1;
    r.V = X;
    r.AV = AV;
    r.BV = BV;
    r.SV = SV;
    r.ready = ev_ready_;
    r.done = ev_done_;
    PPW_HIP(hipEventRecord(ev_ready_, s_));
    pb_->multiply(r);
    PPW_HIP(hipStreamWaitEvent(s_, ev_done_, 0));
    products_ += k;
  }

  // symmetric orthonormalization of the kk vectors in X ([kk][N]); keeps eigen-directions of
  // the Gram matrix above thresh. Returns kept count; X <- X T, R (nk x kk, ld kk) such that
  // X_old ~= X_new R.
  int sym_orth(double* X, int kk, double thresh, double* Xout) {
    tn(kk, kk, X, X, g_, kk);
    symmetrize_kernel<<<gridn((long)kk * kk), kB, 0, s_>>>(g_, kk);
    small_syev(kk, g_, lam_, U_, s_, eigscr_);
    auto lam = fetch(lam_, kk);
    std::vector<int> keep;
    for (int j = 0; j < kk; ++j)
      if (lam[j] > thresh) keep.push_back(j);
    const int nk = (int)keep.size();
    if (nk == 0) return 0;
    upload(keep_, keep);
    symorth_factors_kernel<<<gridn((long)kk * nk), kB, 0, s_>>>(kk, U_, lam_, keep_, nk, Tm_, Rm_);
    // Xout[jj][r] = sum_j T[j][jj] X[j][r]
    expand(nk, kk, Tm_, nk, X, Xout);
    return nk;
  }

  // Add span(X) ([kk][N]) to the basis.  On return the coefficients of the input
  // vectors in the extended basis are in Ctot_ ([nb_new][kk], ld kk).
  int extend(double* X, int kk) {
    const int nb0 = nb_;
    column_dots(X, X, N_, kk, nrm_, s_);
    sqrt_kernel<<<1, kB, 0, s_>>>(nrm_, kk);
    auto nr = fetch(nrm_, kk);
    for (double& x : nr)
      if (!(x > 0)) x = 1.0;
    upload(nrm_, nr);
    scale_rows_kernel<<<gridn(N_ * kk), kB, 0, s_>>>(X, N_, kk, nrm_, 1);
    // pass 1: C1 = Q X^T, X -= C1^T Q
    if (nb0) {
      tn(nb0, kk, Q_, X, c1_, kk);
      expand(kk, nb0, c1_, kk, Q_, X, -1.0, 1.0);
    }
    int n1 = sym_orth(X, kk, 1e-12, T1_);
    if (n1 == 0) {
      // nothing new: coefficients are C1 only
      small_copy_coeffs(nb0, kk, nb0 ? c1_ : nullptr, nullptr, 0, nr);
      return 0;
    }
    // R1 (n1 x kk) saved
    PPW_HIP(hipMemcpyAsync(Rtot_, Rm_, sizeof(double) * n1 * kk, hipMemcpyDeviceToDevice, s_));
    // pass 2
    if (nb0) {
      tn(nb0, n1, Q_, T1_, c2_, n1);
      expand(n1, nb0, c2_, n1, Q_, T1_, -1.0, 1.0);
    }
    int n2 = sym_orth(T1_, n1, 0.25, Q_ + (size_t)nb0 * N_);
    // coefficient rows for the new vectors: R = R2 R1 (n2 x kk)
    if (n2 > 0) small_mm(n2, kk, n1, Rm_, n1, 0, Rtot_, kk, 0, tmp2_, kk);
    // C = C1 + C2 R1 (nb0 x kk)
    if (nb0) {
      PPW_HIP(hipMemcpyAsync(Ctot_, c1_, sizeof(double) * nb0 * kk, hipMemcpyDeviceToDevice, s_));
      small_mm(nb0, kk, n1, c2_, n1, 0, Rtot_, kk, 0, Ctot_, kk, 1.0, 1.0);
    }
    if (n2 > 0) PPW_HIP(hipMemcpyAsync(Ctot_ + (size_t)nb0 * kk, tmp2_, sizeof(double) * n2 * kk,
                                       hipMemcpyDeviceToDevice, s_));
    // undo the unit scaling: column j of C times nrm[j]
    scale_cols_kernel<<<gridn((long)(nb0 + n2) * kk), kB, 0, s_>>>(Ctot_, nb0 + n2, kk, kk, nrm_, 0);
    // products of the new orthonormal vectors
    if (n2 > 0) {
      products(n2, Q_ + (size_t)nb0 * N_, false);
      axpby((long)n2 * N_, 1.0, AV_, 0.0, P0_ + (size_t)nb0 * N_, s_);
      axpby((long)n2 * N_, 1.0, BV_, 1.0, P0_ + (size_t)nb0 * N_, s_);
      axpby((long)n2 * N_, 1.0, AV_, 0.0, P1_ + (size_t)nb0 * N_, s_);
      axpby((long)n2 * N_, -1.0, BV_, 1.0, P1_ + (size_t)nb0 * N_, s_);
      PPW_HIP(hipMemcpyAsync(PS_ + (size_t)nb0 * N_, SV_, sizeof(double) * n2 * N_, hipMemcpyDeviceToDevice, s_));
    }
    nb_ = nb0 + n2;
    return n2;
  }

  void small_copy_coeffs(int nb0, int kk, const double* c1, const double*, int, const std::vector<double>&) {
    if (nb0) {
      PPW_HIP(hipMemcpyAsync(Ctot_, c1, sizeof(double) * nb0 * kk, hipMemcpyDeviceToDevice, s_));
      scale_cols_kernel<<<gridn((long)nb0 * kk), kB, 0, s_>>>(Ctot_, nb0, kk, kk, nrm_, 0);
    }
  }

  // Zt, Zb (in T3_, T4_) for block coefficient vectors cx, cy (nb_ x k, ld kmax_)
  void zprod(int k, const double* cx, const double* cy, double* Zt, double* Zb) {
    // cu = cx + cy, cw = cx - cy
    PPW_HIP(hipMemcpyAsync(cu_, cx, sizeof(double) * nbmax_ * kmax_, hipMemcpyDeviceToDevice, s_));
    PPW_HIP(hipMemcpyAsync(cw_, cx, sizeof(double) * nbmax_ * kmax_, hipMemcpyDeviceToDevice, s_));
    axpby((long)nbmax_ * kmax_, 1.0, cy, 1.0, cu_, s_);
    axpby((long)nbmax_ * kmax_, -1.0, cy, 1.0, cw_, s_);
    expand(k, nb_, cu_, kmax_, P0_, T1_);   // PU
    expand(k, nb_, cw_, kmax_, P1_, T2_);   // MW
    expand(k, nb_, cx, kmax_, PS_, T5_);    // SX
    expand(k, nb_, cy, kmax_, PS_, T6_);    // SY
    zcombine_kernel<<<gridn(N_ * k), kB, 0, s_>>>(N_ * k, w0_, T1_, T2_, T5_, T6_, Zt, Zb);
  }

  void two_dots(const double* A1, const double* B1, const double* A2, const double* B2, long N, int k, double* out) {
    two_dots_kernel<<<k, kB, 0, s_>>>(A1, B1, A2, B2, N, out);
  }
  void coeff_dots(int k, const double* X1, const double* Y1, const double* X2, const double* Y2, double* out) {
    coeff_dots_kernel<<<(k + 63) / 64, 64, 0, s_>>>(nb_, k, kmax_, X1, Y1, X2, Y2, out);
  }

  // thick restart: new basis = orthonormal span of the X+Y and X-Y halves of the block's Ritz vectors
  void restart(const std::vector<int>& blk) {
    const int n = nb_;
    const int b = (int)blk.size();
    const int kk = 2 * b;
    std::vector<int> cols(blk);
    upload(sel_, cols);
    gather_cols_kernel<<<gridn((long)n * b), kB, 0, s_>>>(n, b, sel_, us_, rld_, tmp_, kk, 0);
    gather_cols_kernel<<<gridn((long)n * b), kB, 0, s_>>>(n, b, sel_, ws_, rld_, tmp_, kk, b);
    // Gram of the coefficient vectors (n rows) and symmetric orthonormalization
    small_mm(kk, kk, n, tmp_, kk, 1, tmp_, kk, 0, g_, kk);
    symmetrize_kernel<<<gridn((long)kk * kk), kB, 0, s_>>>(g_, kk);
    small_syev(kk, g_, lam_, U_, s_, eigscr_);
    auto lam = fetch(lam_, kk);
    std::vector<int> keep;
    for (int j = 0; j < kk; ++j)
      if (lam[j] > 1e-12 * std::max(1.0, lam[kk - 1])) keep.push_back(j);
    const int nk = (int)keep.size();
    upload(keep_, keep);
    symorth_factors_kernel<<<gridn((long)kk * nk), kB, 0, s_>>>(kk, U_, lam_, keep_, nk, Tm_, Rm_);
    // Kc = tmp T  (n x nk)
    small_mm(n, nk, kk, tmp_, kk, 0, Tm_, nk, 0, tmp2_, nk);
    expand(nk, n, tmp2_, nk, Q_, Qs_);
    if (opt_.precision == 1) {
      // mixed precision: the restart block gets FP64 products (refinement)
      products(nk, Qs_, true);
      axpby((long)nk * N_, 1.0, AV_, 0.0, P0s_, s_);
      axpby((long)nk * N_, 1.0, BV_, 1.0, P0s_, s_);
      axpby((long)nk * N_, 1.0, AV_, 0.0, P1s_, s_);
      axpby((long)nk * N_, -1.0, BV_, 1.0, P1s_, s_);
      PPW_HIP(hipMemcpyAsync(PSs_, SV_, sizeof(double) * nk * N_, hipMemcpyDeviceToDevice, s_));
    } else {
      expand(nk, n, tmp2_, nk, P0_, P0s_);
      expand(nk, n, tmp2_, nk, P1_, P1s_);
      expand(nk, n, tmp2_, nk, PS_, PSs_);
    }
    std::swap(Q_, Qs_);
    std::swap(P0_, P0s_);
    std::swap(P1_, P1s_);
    std::swap(PS_, PSs_);
    nb_ = nk;
  }

  // Riesz projector mode: V_ (X rows [0, k), Y rows [k, 2k)) <- P V_ on the circle of
  // radius rad_ around omega0
  void contour_step(int k) {
    ContourParams p;
    p.center = w0_;
    p.radius = rad_;
    p.nodes = opt_.contour_nodes;
    // shifted solves: contour_tol on the first cycle, then a tenth of the window's worst
    // residual (the filtered subspace is only as accurate as the solves), down to a
    // tenth of the solver tolerance (FP32 products: not below 1e-6)
    const double floor_tol = (opt_.precision == 1 && !refined_) ? 1e-6 : 0.1 * opt_.tol;
    p.tol = std::max(floor_tol, std::min(opt_.contour_tol, 0.1 * contour_worst_));
    p.maxit = opt_.contour_maxit;
    double worst = 0.0;
    const int it = cf_->apply(p, k, V_, [this](int kc, const double* X, double* AV, double* BV, double* SV) {
      products_into(kc, X, AV, BV, SV, false);
    }, &worst);
    contour_iters_ += it;
    if (trace_)
      std::fprintf(stderr, "[ppwin] window %d contour radius %.3e: %d vectors, %d iterations, residual %.2e\n", id_,
                   rad_, k, it, worst);
  }
  // V_ <- X and Y halves of the Ritz vectors listed in act (from the current basis)
  void ritz_block(const std::vector<int>& act) {
    const int k = (int)act.size(), n = nb_;
    upload(sel_, act);
    gather_cols_kernel<<<gridn((long)n * k), kB, 0, s_>>>(n, k, sel_, us_, rld_, c1_, k, 0);
    gather_cols_kernel<<<gridn((long)n * k), kB, 0, s_>>>(n, k, sel_, ws_, rld_, c2_, k, 0);
    expand(k, n, c1_, k, Q_, T1_);
    expand(k, n, c2_, k, Q_, T2_);
    halves_kernel<<<gridn(N_ * k), kB, 0, s_>>>(N_ * k, T1_, T2_, V_, V_ + (size_t)k * N_);
  }

  struct Ritz {
    std::vector<double> th, rn, fold;
  };
  Ritz rayleigh_ritz();
};

Solver::Ritz Solver::rayleigh_ritz() {
  const int n = nb_;
  tn(n, n, Q_, P0_, Ap_, n);
  tn(n, n, Q_, P1_, Am_, n);
  tn(n, n, Q_, PS_, Sp_, n);
  symmetrize_kernel<<<gridn((long)n * n), kB, 0, s_>>>(Ap_, n);
  symmetrize_kernel<<<gridn((long)n * n), kB, 0, s_>>>(Am_, n);
  symmetrize_kernel<<<gridn((long)n * n), kB, 0, s_>>>(Sp_, n);
  small_cholesky(n, Am_, L_, ival_, s_);
  // Sp^-1: the metric is the identity plus the (small) MP2 density correction, so
  // Newton-Schulz X <- 2X - X Sp X from X = I converges quadratically; the Cholesky
  // route is the fallback when |I - Sp X| does not reach rounding level.
  identity_kernel<<<gridn((long)n * n), kB, 0, s_>>>(Spi_, n);
  if (c_.order >= 2) {
    for (int it = 0; it < 6; ++it) {
      small_mm(n, n, n, Sp_, n, 0, Spi_, n, 0, tmp_, n);        // T = Sp X
      small_mm(n, n, n, Spi_, n, 0, tmp_, n, 0, tmp2_, n);      // X T
      axpby((long)n * n, 2.0, Spi_, 0.0, K_, s_);               // 2X
      axpby((long)n * n, -1.0, tmp2_, 1.0, K_, s_);             // 2X - X T
      PPW_HIP(hipMemcpyAsync(Spi_, K_, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s_));
    }
    small_mm(n, n, n, Sp_, n, 0, Spi_, n, 0, tmp_, n);
    ns_residual_kernel<<<1, 256, 0, s_>>>(n, tmp_, lam_);
  }
  auto info = fetch(ival_, 1);
  if (info[0] != 0) throw Unstable("A - B is not positive definite in the subspace");
  if (c_.order >= 2) {
    auto res = fetch(lam_, 1);
    if (!(res[0] < 1e-13)) {
      small_cholesky(n, Sp_, Ls_, ival_ + 1, s_);
      auto inf2 = fetch(ival_ + 1, 1);
      if (inf2[0] != 0) throw Unstable("S is not positive definite in the subspace");
      small_trinv(n, Ls_, Lsi_, s_);
      small_mm(n, n, n, Lsi_, n, 1, Lsi_, n, 0, Spi_, n);
    }
  }
  // Mt = Sp^-1 L ; K = Mt^T Ap Mt
  small_mm(n, n, n, Spi_, n, 0, L_, n, 0, tmp_, n);
  small_mm(n, n, n, Ap_, n, 0, tmp_, n, 0, tmp2_, n);
  small_mm(n, n, n, tmp_, n, 1, tmp2_, n, 0, K_, n);
  symmetrize_kernel<<<gridn((long)n * n), kB, 0, s_>>>(K_, n);
  // eigenpairs of K nearest omega0^2 (candidate roots of the window)
  const int p = std::min(n, std::min(64, std::max(2 * m_ + 4, nr_ + 8)));
  const int q = partial_syev(n, K_, w0_ * w0_, p, th2_, Zk_, eigscr_, s_);
  auto th2 = fetch(th2_, q);
  for (int j = 0; j < q; ++j)
    if (!(th2[j] > 0)) throw Unstable("A + B is not positive definite in the subspace");
  std::vector<double> th(q);
  for (int j = 0; j < q; ++j) th[j] = std::sqrt(th2[j]);
  upload(th_, th);
  rld_ = q;
  // us = Mt Z / sqrt(theta),  ws = sqrt(theta) L^-T Z
  small_mm(n, q, n, tmp_, n, 0, Zk_, p, 0, us_, q);
  scale_cols_kernel<<<gridn((long)n * q), kB, 0, s_>>>(us_, n, q, q, th_, 3);
  copy_cols_kernel<<<gridn((long)n * q), kB, 0, s_>>>(n, q, Zk_, p, ws_, q);
  small_trsm_lt(n, L_, q, ws_, s_);
  scale_cols_kernel<<<gridn((long)n * q), kB, 0, s_>>>(ws_, n, q, q, th_, 2);
  // products of the Ritz halves: PU = P0 us, MW = P1 ws, SU = PS us, SW = PS ws  ([q][N])
  expand(q, n, us_, q, P0_, RU_);
  expand(q, n, ws_, q, P1_, RW_);
  expand(q, n, us_, q, PS_, RSU_);
  expand(q, n, ws_, q, PS_, RSW_);
  residual_norms_kernel<<<q, kB, 0, s_>>>(N_, q, th_, w0_, RU_, RW_, RSU_, RSW_, stats_);
  coeff_norms_kernel<<<(q + 63) / 64, 64, 0, s_>>>(n, q, us_, ws_, stats_ + 2 * q);
  auto st = fetch(stats_, 3 * (size_t)q);
  Ritz R;
  R.th = th;
  R.rn.resize(q);
  R.fold.resize(q);
  for (int j = 0; j < q; ++j) {
    const double y2 = 0.5 * st[2 * q + j];   // |y|^2 = (|u|^2 + |w|^2)/2, Q orthonormal
    R.rn[j] = std::sqrt(0.5 * st[j] / y2);
    R.fold[j] = 0.5 * st[q + j] / y2;
  }
  return R;
}

void Solver::run(double* energies, double* vectors, double* osc, pp_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  // start block: m top-half pairs with the smallest |A_ii - w0 S_ii|
  auto dA = fetch(c_.dA, N_);
  auto dS = fetch(c_.dS, N_);
  std::vector<long> idx(N_);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](long a, long b) {
    return std::fabs(dA[a] - w0_ * dS[a]) < std::fabs(dA[b] - w0_ * dS[b]);
  });
  std::vector<int> pos(m_);
  for (int q = 0; q < m_; ++q) pos[q] = (int)idx[q];
  std::mt19937_64 rng(opt_.seed ^ 0x9e3779b97f4a7c15ULL);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> noise((size_t)2 * m_ * N_);
  for (double& x : noise) x = nd(rng);
  upload(noise_, noise);
  upload(sel_, pos);
  start_block_kernel<<<gridn(N_ * m_), kB, 0, s_>>>(N_, m_, sel_, noise_, V_, V_ + (size_t)m_ * N_);
  if (cf_) {
    // first circle from the zeroth-order picture: the diagonal estimates A_ii / S_ii
    std::vector<double> d(N_);
    for (long i = 0; i < N_; ++i) d[i] = std::fabs(dA[i] / dS[i] - w0_);
    std::sort(d.begin(), d.end());
    rad_ = 1.5 * d[std::min<long>(nr_, N_) - 1] + 1e-6;
  }

  int knew = m_;  // columns in the new block (X in V_[0..k), Y in V_[k..2k))
  Ritz R;
  std::vector<int> tgt, blk, inner, out;
  bool converged = false;
  int cycle = 0;
  const double clampv = opt_.d_clamp > 0 ? opt_.d_clamp : 1e-4;
  const bool mixed = opt_.precision == 1;
  bool refined = !mixed;  // mixed precision: becomes true after the first FP64 restart
  const double switch_tol = std::max(opt_.tol, 1e-7);
  double best_worst = 1e300;
  int since_best = 0;
  for (cycle = 0; cycle < opt_.max_cycles; ++cycle) {
   if (knew > 0 && cf_) {
    // Riesz projector mode (subspace iteration): the filtered block replaces the subspace
    contour_step(knew);
    nb_ = 0;
    extend(V_, 2 * knew);
   } else if (knew > 0) {
    // X, Y halves are contiguous in V_: [X_0..X_k-1, Y_0..Y_k-1]
    const int kk = 2 * knew;
    extend(V_, kk);
    // coefficients of X_q (col q) and Y_q (col k+q) in Ctot_ (nb_ x kk, ld kk)
    PPW_HIP(hipMemsetAsync(cx_, 0, sizeof(double) * nbmax_ * kmax_, s_));
    PPW_HIP(hipMemsetAsync(cy_, 0, sizeof(double) * nbmax_ * kmax_, s_));
    {
      std::vector<int> a(knew), b(knew);
      for (int q = 0; q < knew; ++q) {
        a[q] = q;
        b[q] = knew + q;
      }
      upload(sel_, a);
      gather_cols_kernel<<<gridn((long)nb_ * knew), kB, 0, s_>>>(nb_, knew, sel_, Ctot_, kk, cx_, kmax_, 0);
      upload(sel_, b);
      gather_cols_kernel<<<gridn((long)nb_ * knew), kB, 0, s_>>>(nb_, knew, sel_, Ctot_, kk, cy_, kmax_, 0);
    }
    for (int st = 1; st < opt_.krylov_steps; ++st) {
      if (nb_ + kk > nbmax_) break;
      zprod(knew, cx_, cy_, T3_, T4_);
      expand(knew, nb_, cx_, kmax_, Q_, T1_);
      expand(knew, nb_, cy_, kmax_, Q_, T2_);
      jacobi_dir_kernel<<<gridn(N_ * knew), kB, 0, s_>>>(N_, knew, w0_, clampv, c_.dA, c_.dS, T1_, T2_, T3_, T4_,
                                                          V_, V_ + (size_t)knew * N_);
      // keep Zt, Zb of the current z
      PPW_HIP(hipMemcpyAsync(T5_, T3_, sizeof(double) * knew * N_, hipMemcpyDeviceToDevice, s_));
      PPW_HIP(hipMemcpyAsync(T6_, T4_, sizeof(double) * knew * N_, hipMemcpyDeviceToDevice, s_));
      extend(V_, kk);
      PPW_HIP(hipMemsetAsync(cdx_, 0, sizeof(double) * nbmax_ * kmax_, s_));
      PPW_HIP(hipMemsetAsync(cdy_, 0, sizeof(double) * nbmax_ * kmax_, s_));
      {
        std::vector<int> a(knew), b(knew);
        for (int q = 0; q < knew; ++q) {
          a[q] = q;
          b[q] = knew + q;
        }
        upload(sel_, a);
        gather_cols_kernel<<<gridn((long)nb_ * knew), kB, 0, s_>>>(nb_, knew, sel_, Ctot_, kk, cdx_, kmax_, 0);
        upload(sel_, b);
        gather_cols_kernel<<<gridn((long)nb_ * knew), kB, 0, s_>>>(nb_, knew, sel_, Ctot_, kk, cdy_, kmax_, 0);
      }
      // Zd in T3_, T4_ (Zt, Zb of z kept in T5_, T6_: unchanged by the basis extension)
      PPW_HIP(hipMemcpyAsync(T1_, T5_, sizeof(double) * knew * N_, hipMemcpyDeviceToDevice, s_));
      PPW_HIP(hipMemcpyAsync(T2_, T6_, sizeof(double) * knew * N_, hipMemcpyDeviceToDevice, s_));
      // T1_/T2_ now hold Zt/Zb; zprod overwrites T1_, T2_, T5_, T6_ -> move Zt/Zb to AV_/BV_
      PPW_HIP(hipMemcpyAsync(AV_, T1_, sizeof(double) * knew * N_, hipMemcpyDeviceToDevice, s_));
      PPW_HIP(hipMemcpyAsync(BV_, T2_, sizeof(double) * knew * N_, hipMemcpyDeviceToDevice, s_));
      zprod(knew, cdx_, cdy_, T3_, T4_);
      // stats: [0] |Zz|^2, [1] Zz.Zd, [2] |Zd|^2, [3] c.cd, [4] |cd|^2, [5] |c|^2
      two_dots(AV_, BV_, AV_, BV_, N_, knew, st_ + 0 * knew);
      two_dots(AV_, BV_, T3_, T4_, N_, knew, st_ + 1 * knew);
      two_dots(T3_, T4_, T3_, T4_, N_, knew, st_ + 2 * knew);
      coeff_dots(knew, cx_, cy_, cdx_, cdy_, st_ + 3 * knew);
      coeff_dots(knew, cdx_, cdy_, cdx_, cdy_, st_ + 4 * knew);
      coeff_dots(knew, cx_, cy_, cx_, cy_, st_ + 5 * knew);
      alpha_kernel<<<1, 64, 0, s_>>>(knew, st_, alpha_);
      axpy_cols_kernel<<<gridn((long)nb_ * knew), kB, 0, s_>>>(nb_, knew, kmax_, alpha_, cdx_, kmax_, cx_);
      axpy_cols_kernel<<<gridn((long)nb_ * knew), kB, 0, s_>>>(nb_, knew, kmax_, alpha_, cdy_, kmax_, cy_);
    }
   }
    R = rayleigh_ritz();
    const int n = (int)R.th.size();
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return R.fold[a] < R.fold[b]; });
    // targets: the n_roots pairs with the smallest folded quotient.  Every Ritz pair
    // whose value lies within the farthest target's distance of omega0 ("inner") must
    // converge too: an eigenvector already in the subspace can show up as a polluted
    // Ritz pair (large residual, large folded quotient) next to omega0, and would
    // otherwise be dropped at a restart while farther roots converge.  The inner pairs
    // lead the block, so they get corrections and survive restarts.
    bool all = false;
    double worst = 0.0;
    if (cf_) {
      // Riesz mode: the subspace is the filtered block's X and Y halves, and its paired
      // closure holds directions the filter never touched; they give Ritz pairs that do
      // not converge (residual of order one) and can sit nearer omega0 than true roots.
      // The window is taken among the pairs whose residual is below 1e-2 (a true
      // eigenvector inside the contour is in the filtered span, so its Ritz pair
      // converges): the n_roots nearest of them, all of which must meet the tolerance.
      std::vector<int> byd(n), rel;
      std::iota(byd.begin(), byd.end(), 0);
      std::stable_sort(byd.begin(), byd.end(),
                       [&](int a, int b) { return std::fabs(R.th[a] - w0_) < std::fabs(R.th[b] - w0_); });
      for (int j : byd)
        if (R.rn[j] <= 1e-2) rel.push_back(j);
      const bool enough = (int)rel.size() >= nr_;
      const std::vector<int>& src = enough ? rel : byd;
      out.assign(src.begin(), src.begin() + std::min<int>(nr_, (int)src.size()));
      tgt = out;
      inner = out;
      all = enough && (int)out.size() == nr_;
      for (int j : out) {
        all = all && R.rn[j] <= opt_.tol;
        worst = std::max(worst, R.rn[j]);
      }
      // block: the reliable pairs first (nearest first), then the rest by distance
      blk.clear();
      for (int j : rel)
        if ((int)blk.size() < m_) blk.push_back(j);
      for (int j : byd) {
        if ((int)blk.size() >= std::min(m_, n)) break;
        if (std::find(blk.begin(), blk.end(), j) == blk.end()) blk.push_back(j);
      }
      // the circle passes halfway between the window's farthest pair and the next one
      // (reliable pairs when there are enough of them)
      const std::vector<int>& dref = (int)rel.size() > nr_ ? rel : byd;
      if ((int)dref.size() > nr_)
        rad_ = 0.5 * (std::fabs(R.th[dref[nr_ - 1]] - w0_) + std::fabs(R.th[dref[nr_]] - w0_));
      else if (!dref.empty())
        rad_ = 1.25 * std::fabs(R.th[dref.back()] - w0_);
      rad_ = std::max(rad_, 1e-8);
    } else {
    tgt.assign(order.begin(), order.begin() + std::min(nr_, n));
    double dmax = 0.0;
    for (int j : tgt) dmax = std::max(dmax, std::fabs(R.th[j] - w0_));
    inner.clear();
    for (int j = 0; j < n; ++j)
      if (std::fabs(R.th[j] - w0_) <= dmax * (1.0 + 1e-12)) inner.push_back(j);
    std::stable_sort(inner.begin(), inner.end(),
                     [&](int a, int b) { return std::fabs(R.th[a] - w0_) < std::fabs(R.th[b] - w0_); });
    blk.clear();
    for (int j : inner)
      if ((int)blk.size() < m_) blk.push_back(j);
    for (int j : order) {
      if ((int)blk.size() >= std::min(m_, n)) break;
      if (std::find(blk.begin(), blk.end(), j) == blk.end()) blk.push_back(j);
    }
    all = (int)tgt.size() == nr_;
    for (int j : tgt) {
      all = all && R.rn[j] <= opt_.tol;
      worst = std::max(worst, R.rn[j]);
    }
    for (int j : inner) {
      all = all && R.rn[j] <= opt_.tol;
      worst = std::max(worst, R.rn[j]);
    }
    // the window's result: the n_roots inner pairs nearest omega0 (the targets while
    // some inner pair is unresolved)
    if ((int)inner.size() >= nr_) out.assign(inner.begin(), inner.begin() + nr_);
    else out = tgt;
    }
    if (worst < 0.5 * best_worst) {
      best_worst = worst;
      since_best = 0;
    } else {
      ++since_best;
    }
    const bool stalled = since_best >= 5;
    if (trace_)
      std::fprintf(stderr, "[ppwin] window %d omega0 %.4f cycle %d basis %d products %ld worst %.3e refined %d\n", id_,
                   w0_, cycle, nb_, products_, worst, refined ? 1 : 0);
    if (mixed) {
      // Reduced-precision products build the subspace until the window is resolved to
      // that level (or stops improving); then a thick restart onto the block with FP64
      // products, and the solve continues as in FP64 (every later product FP64); the
      // returned vectors are accepted on residuals of FP64 products only.
      if (!refined && (all || worst <= switch_tol || stalled)) {
        // thick restart onto the block (inner pairs first): only its X+Y and X-Y halves
        // get FP64 products, and every later product is FP64
        refined_ = true;
        restart(blk);
        refined = true;
        knew = 0;
        best_worst = 1e300;
        since_best = 0;
        continue;
      }
      if (refined && all) {
        // every basis product since the switch is FP64, so these Rayleigh-Ritz residuals
        // are residuals of FP64 products
        converged = true;
        ++cycle;
        break;
      }
    } else if (all) {
      converged = true;
      ++cycle;
      break;
    }
    // corrections for the block's unconverged pairs; after the precision switch of a
    // mixed solve only for the targets and inner pairs (the Ritz vectors already hold
    // the reduced-precision solution, and the guard pairs' FP64 products cost more than
    // they speed up the targets)
    std::vector<int> act;
    for (int j : blk) {
      if (R.rn[j] <= opt_.tol) continue;
      if (mixed && refined && !cf_ && std::find(inner.begin(), inner.end(), j) == inner.end() &&
          std::find(tgt.begin(), tgt.end(), j) == tgt.end())
        continue;
      act.push_back(j);
    }
    if (act.empty()) act = blk;
    knew = (int)act.size();
    upload(sel_, act);
    // corrections into V_ (X part then Y part); residual vectors are in RU_/RW_
    if (cf_) {
      // Riesz mode: the next block is the block's Ritz vectors, filtered at the start of
      // the next cycle; solves are tightened as the window converges
      knew = (int)blk.size();
      ritz_block(blk);
      contour_worst_ = worst;
    } else {
      correction_kernel<<<gridn(N_ * knew), kB, 0, s_>>>(N_, knew, sel_, th_, clampv, c_.dA, c_.dB, c_.dS, RU_, RW_,
                                                          V_, V_ + (size_t)knew * N_);
      if (nb_ + 2 * opt_.krylov_steps * knew > nbmax_) restart(blk);
    }
  }
  // outputs: the window's roots, ascending energy
  std::vector<int> sel = out;
  std::sort(sel.begin(), sel.end(), [&](int a, int b) { return R.th[a] < R.th[b]; });
  const int r = (int)sel.size();
  for (int q = 0; q < r; ++q) energies[q] = R.th[sel[q]];
  upload(sel_, sel);
  const int n = nb_;
  // coefficient columns of the selected roots: us_sel, ws_sel ([n][r], ld r)
  gather_cols_kernel<<<gridn((long)n * r), kB, 0, s_>>>(n, r, sel_, us_, rld_, c1_, r, 0);
  gather_cols_kernel<<<gridn((long)n * r), kB, 0, s_>>>(n, r, sel_, ws_, rld_, c2_, r, 0);
  expand(r, n, c1_, r, Q_, T1_);
  expand(r, n, c2_, r, Q_, T2_);
  if (vectors) {
    pair_out_kernel<<<gridn(2 * N_ * r), kB, 0, s_>>>(N_, r, T1_, T2_, T3_);
    PPW_HIP(hipMemcpyAsync(vectors, T3_, sizeof(double) * 2 * N_ * r, hipMemcpyDeviceToHost, s_));
  }
  if (osc) {
    // T[x][j] = sum_ia dip[x][ia] u_j[ia]
    const double* F = (opt_.correlated_f && c_.dipS) ? c_.dipS : c_.dip;
    gemm(gd(3, r, (int)N_, 0, N_, 1, N_, r), 1.0, F, T1_, 0.0, tmp_);
    std::vector<double> thsel(r);
    for (int q = 0; q < r; ++q) thsel[q] = R.th[sel[q]];
    upload(th2_, thsel);
    osc_kernel<<<1, 64, 0, s_>>>(r, tmp_, th2_, lam_);
    auto f = fetch(lam_, r);
    for (int q = 0; q < r; ++q) osc[q] = f[q];
  }
  PPW_HIP(hipStreamSynchronize(s_));
  if (info) {
    info->cycles = cycle;
    info->basis = nb_;
    info->products = products_;
    info->n_roots = r;
    for (int q = 0; q < r && q < PP_MAX_ROOTS; ++q) {
      info->residual[q] = R.rn[sel[q]];
      info->converged[q] = R.rn[sel[q]] <= opt_.tol ? 1 : 0;
    }
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!converged) throw NotConverged("window solve reached max_cycles before every root met the tolerance");
}


}  // namespace

void window_solve_many(Context& c, const SolveOptions& opt, int nw, const double* omega0, int n_roots,
                       double* energies, double* vectors, double* osc, pp_solve_info* info) {
  PPW_HIP(hipSetDevice(c.device));
  if (nw < 1) return;
  c.resolve_stats();
  const double sig0 = c.stats.seconds, flop0 = c.stats.flops;
  // Two groups of windows (even and odd index) with passes of their own: while one
  // group's pass runs, the other group's windows solve their projected problems, so
  // the product stream does not wait for every window's subspace work.  Group
  // membership is fixed, so every pass (and every result) is reproducible.
  const int ngroups = nw >= 2 ? 2 : 1;
  std::mutex enqueue;
  std::vector<std::unique_ptr<ProductBatcher>> pbs;
  for (int g = 0; g < ngroups; ++g) {
    int members = 0;
    for (int w = g; w < nw; w += ngroups) ++members;
    pbs.emplace_back(new ProductBatcher(c, members, opt.precision, &enqueue, opt.pass_vectors));
  }
  std::vector<std::unique_ptr<Solver>> sv;
  std::vector<int> ktot(ngroups, 0);
  for (int w = 0; w < nw; ++w) {
    sv.emplace_back(new Solver(c, opt, omega0[w], n_roots, pbs[w % ngroups].get(), w));
    ktot[w % ngroups] += sv.back()->kmax();
  }
  for (int g = 0; g < ngroups; ++g) pbs[g]->reserve(ktot[g]);
  PPW_HIP(hipStreamSynchronize(c.stream));
  std::vector<std::exception_ptr> errs(nw);
  auto work = [&](int w) {
    try {
      PPW_HIP(hipSetDevice(c.device));
      const size_t N = (size_t)c.N;
      sv[w]->run(energies + (size_t)w * n_roots, vectors ? vectors + (size_t)w * n_roots * 2 * N : nullptr,
                 osc ? osc + (size_t)w * n_roots : nullptr, info ? info + w : nullptr);
    } catch (...) {
      errs[w] = std::current_exception();
    }
    pbs[w % ngroups]->leave();
  };
  if (nw == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w) th.emplace_back(work, w);
    for (auto& t : th) t.join();
  }
  PPW_HIP(hipStreamSynchronize(c.stream));
  sv.clear();
  c.resolve_stats();
  if (info)
    for (int w = 0; w < nw; ++w) {
      info[w].sigma_seconds = c.stats.seconds - sig0;
      info[w].sigma_flops = c.stats.flops - flop0;
    }
  std::exception_ptr notconv;
  for (auto& e : errs) {
    if (!e) continue;
    try {
      std::rethrow_exception(e);
    } catch (const NotConverged&) {
      notconv = e;
    }
  }
  if (notconv) std::rethrow_exception(notconv);
}

void window_solve(Context& c, const SolveOptions& opt, double omega0, int n_roots, double* energies,
                  double* vectors, double* osc, pp_solve_info* info) {
  window_solve_many(c, opt, 1, &omega0, n_roots, energies, vectors, osc, info);
}


int window_block_vectors(long N, int n_roots, const SolveOptions& opt) { return solver_dims(N, n_roots, opt).kmax; }

size_t window_solve_bytes(long N, int n_roots, const SolveOptions& opt) {
  // mirrors Solver::alloc (arena blocks are rounded to 256 B)
  const SolverDims d = solver_dims(N, n_roots, opt);
  auto r = [](size_t bytes) { return ((bytes + 255) / 256) * 256; };
  const size_t D = sizeof(double);
  const size_t bN = (size_t)d.nbmax * N, kN = (size_t)d.kmax * N;
  const size_t bk = (size_t)d.nbmax * d.kmax, bb = (size_t)d.nbmax * d.nbmax, kk = (size_t)d.kmax * d.kmax;
  size_t t = 12 * r(bN * D) + 10 * r(kN * D);
  t += 2 * r(bk * D);                                   // c1, c2
  t += 2 * r(std::max(kk, bb) * D);                     // gram, eigvec
  t += r(d.nbmax * D);                                  // eigval
  t += r(std::max(kk, bk) * D) + r(kk * D);             // T, R
  t += r(bk * D) + r(kk * D);                           // C, R tot
  t += 2 * r(std::max(bk, bb) * D);                     // tmp, tmp2
  t += r(std::max(d.kmax, 8) * D);                      // norms
  t += 6 * r(bk * D);                                   // cx, cy, cdx, cdy, cu, cw
  t += r((size_t)8 * d.kmax * D) + r((size_t)d.kmax * D);  // stats, alpha
  t += 9 * r(bb * D);                                   // Ap .. K
  t += r(d.nbmax * D) + r(bb * D) + 2 * r(bb * D) + r(d.nbmax * D);  // theta2, Zk, us, ws, theta
  t += r(std::max((size_t)2 * d.nbmax, (size_t)3 * 64) * D);
  t += r(std::max((size_t)2 * std::max(bb, kk), partial_syev_scratch(d.nbmax, 64)) * D);
  t += 2 * r(std::max(d.kmax, d.nbmax) * sizeof(int)) + r(4 * sizeof(int));
  t += r((size_t)2 * d.m * N * D);                      // noise
  t += r((size_t)32 << 20);                             // split-K workspace
  if (opt.method == 1) t += ContourFilter::bytes(N, d.m, opt.contour_nodes);
  return t;
}

void window_solve_shared(Context& c, const SolveOptions& opt, double omega0, int n_roots, ProductSink& sink, int id,
                         double* energies, double* vectors, double* osc, pp_solve_info* info) {
  PPW_HIP(hipSetDevice(c.device));
  Solver sv(c, opt, omega0, n_roots, &sink, id);
  PPW_HIP(hipStreamSynchronize(c.stream));
  sv.run(energies, vectors, osc, info);
}

}  // namespace ppw
