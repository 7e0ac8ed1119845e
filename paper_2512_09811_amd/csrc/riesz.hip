// Riesz projector on a circular contour (section on the connection to the Riesz
// projector): trapezoidal quadrature of the resolvent of the pencil, each shifted system
// solved by diagonal-preconditioned conjugate-orthogonal CG with the library's products.
//
// For an eigenpair M z = omega Sigma z, (z Sigma - M)^-1 Sigma z = z / (z - omega), so the
// 2n-node rule maps z to rho(x) z with x = (omega - c) / r and rho(x) = 1 / (1 + x^(2n)):
// close to 1 inside the circle, |x|^(-2n) outside.
//
// COCG for a complex symmetric K = z Sigma - M and preconditioner D = diag(K):
//   r = b, u = D^-1 r, p = u, rho = r^T u (bilinear, no conjugation)
//   repeat: q = K p, alpha = rho / p^T q, x += alpha p, r -= alpha q, u = D^-1 r,
//           rho' = r^T u, p = u + (rho' / rho) p
// All systems of one apply advance together; a system stops (alpha = beta = 0) once
// |r| <= tol |b|.  Every vector operation runs on the device; the host reads one residual
// norm per system per iteration to decide when to stop.
#include "riesz.h"

#include <algorithm>
#include <cmath>

namespace ppw {
namespace {

constexpr int kT = 256;
inline int grid_of(long n) { return (int)std::max<long>(1, std::min<long>((n + kT - 1) / kT, 65536)); }

#define CF_LOOP(idx, n) for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (n); idx += (long)gridDim.x * blockDim.x)

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// diagonal of z Sigma - M: top (X) block z dS - dA, bottom (Y) block -z dS - dA
__device__ __forceinline__ cplx diag_top(cplx z, double ds, double da) { return {z.re * ds - da, z.im * ds}; }
__device__ __forceinline__ cplx diag_bot(cplx z, double ds, double da) { return {-z.re * ds - da, -z.im * ds}; }

// Start of every system: x = 0, r = b = Sigma [X_j; Y_j] (top S X_j, bottom -S Y_j, real),
// u = D^-1 r, p = u.  SV rows: S X_0..S X_{k-1}, S Y_0..S Y_{k-1}.
__global__ void cf_init_kernel(long N, int k, int nq, const double* __restrict__ zw, const double* __restrict__ dA,
                               const double* __restrict__ dS, const double* __restrict__ SV, double* __restrict__ X,
                               double* __restrict__ R, double* __restrict__ U, double* __restrict__ P) {
  CF_LOOP(idx, (long)nq * k * N) {
    const long s = idx / N, e = idx % N;
    const int j = (int)(s % k), q = (int)(s / k);
    const cplx z = {zw[4 * q], zw[4 * q + 1]};
    const double bt = SV[(long)j * N + e], bb = -SV[(long)(k + j) * N + e];
    const cplx ut = cdiv({bt, 0.0}, diag_top(z, dS[e], dA[e]));
    const cplx ub = cdiv({bb, 0.0}, diag_bot(z, dS[e], dA[e]));
    const long b = 4 * s * N + e;
    X[b] = 0.0;
    X[b + N] = 0.0;
    X[b + 2 * N] = 0.0;
    X[b + 3 * N] = 0.0;
    R[b] = bt;
    R[b + N] = bb;
    R[b + 2 * N] = 0.0;
    R[b + 3 * N] = 0.0;
    U[b] = ut.re;
    U[b + N] = ub.re;
    U[b + 2 * N] = ut.im;
    U[b + 3 * N] = ub.im;
    P[b] = ut.re;
    P[b + N] = ub.re;
    P[b + 2 * N] = ut.im;
    P[b + 3 * N] = ub.im;
  }
}

// Q = (z Sigma - M) P from the A, B, S products of P's rows:
// M [X; Y] = [A X + B Y; B X + A Y], Sigma [X; Y] = [S X; -S Y].
__global__ void cf_apply_kernel(long N, int k, int nsys, const double* __restrict__ zw, const double* __restrict__ AP,
                                const double* __restrict__ BP, const double* __restrict__ SP, double* __restrict__ Q) {
  CF_LOOP(idx, (long)nsys * N) {
    const long s = idx / N, e = idx % N;
    const int q = (int)(s / k);
    const double zr = zw[4 * q], zi = zw[4 * q + 1];
    const long b = 4 * s * N + e;
    const double axr = AP[b], ayr = AP[b + N], axi = AP[b + 2 * N], ayi = AP[b + 3 * N];
    const double bxr = BP[b], byr = BP[b + N], bxi = BP[b + 2 * N], byi = BP[b + 3 * N];
    const double sxr = SP[b], syr = SP[b + N], sxi = SP[b + 2 * N], syi = SP[b + 3 * N];
    const double mrt = axr + byr, mrb = bxr + ayr, mit = axi + byi, mib = bxi + ayi;
    const double srt = sxr, srb = -syr, sit = sxi, sib = -syi;
    Q[b] = zr * srt - zi * sit - mrt;
    Q[b + N] = zr * srb - zi * sib - mrb;
    Q[b + 2 * N] = zr * sit + zi * srt - mit;
    Q[b + 3 * N] = zr * sib + zi * srb - mib;
  }
}

// One block per system: out[2s..2s+1] = U_s^T W_s (complex bilinear form over the 2N
// entries), herm[s] = |U_s|^2 (if herm is not null).
__global__ void cf_dot_kernel(long N, const double* __restrict__ U, const double* __restrict__ W,
                              double* __restrict__ out, double* __restrict__ herm) {
  __shared__ double red[3][kT / 64];
  const long s = blockIdx.x;
  const long b = 4 * s * N;
  const long n2 = 2 * N;
  double re = 0.0, im = 0.0, h = 0.0;
  for (long i = threadIdx.x; i < n2; i += blockDim.x) {
    const double ur = U[b + i], ui = U[b + n2 + i], wr = W[b + i], wi = W[b + n2 + i];
    re += ur * wr - ui * wi;
    im += ur * wi + ui * wr;
    h += ur * ur + ui * ui;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_down(re, off, 64);
    im += __shfl_down(im, off, 64);
    h += __shfl_down(h, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = re;
    red[1][wave] = im;
    red[2][wave] = h;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0, d = 0.0;
    for (int w = 0; w < kT / 64; ++w) {
      a += red[0][w];
      c += red[1][w];
      d += red[2][w];
    }
    out[2 * s] = a;
    out[2 * s + 1] = c;
    if (herm) herm[s] = d;
  }
}

// alpha_s = rho_s / (p_s^T q_s); zero for a finished system or a vanishing denominator
__global__ void cf_alpha_kernel(int nsys, const double* __restrict__ rho, const double* __restrict__ sig,
                                const int* __restrict__ done, double* __restrict__ alpha) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
    const cplx sg = {sig[2 * s], sig[2 * s + 1]};
    cplx a = {0.0, 0.0};
    if (!done[s] && (sg.re != 0.0 || sg.im != 0.0)) a = cdiv({rho[2 * s], rho[2 * s + 1]}, sg);
    alpha[2 * s] = a.re;
    alpha[2 * s + 1] = a.im;
  }
}

// beta_s = rho'_s / rho_s (zero for a finished system); rho <- rho'
__global__ void cf_beta_kernel(int nsys, double* __restrict__ rho, const double* __restrict__ rho2,
                               const int* __restrict__ done, double* __restrict__ beta) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
    const cplx r0 = {rho[2 * s], rho[2 * s + 1]};
    const cplx r1 = {rho2[2 * s], rho2[2 * s + 1]};
    cplx b = {0.0, 0.0};
    if (!done[s] && (r0.re != 0.0 || r0.im != 0.0)) b = cdiv(r1, r0);
    beta[2 * s] = b.re;
    beta[2 * s + 1] = b.im;
    rho[2 * s] = r1.re;
    rho[2 * s + 1] = r1.im;
  }
}

// x += alpha p, r -= alpha q, u = D^-1 r
__global__ void cf_update_kernel(long N, int k, int nsys, const double* __restrict__ zw, const double* __restrict__ alpha,
                                 const double* __restrict__ dA, const double* __restrict__ dS,
                                 const double* __restrict__ P, const double* __restrict__ Q, double* __restrict__ X,
                                 double* __restrict__ R, double* __restrict__ U) {
  CF_LOOP(idx, (long)nsys * N) {
    const long s = idx / N, e = idx % N;
    const int q = (int)(s / k);
    const cplx z = {zw[4 * q], zw[4 * q + 1]};
    const cplx a = {alpha[2 * s], alpha[2 * s + 1]};
    const long b = 4 * s * N + e;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long re = b + h * N, im = b + 2 * N + h * N;
      const cplx ap = cmul(a, {P[re], P[im]});
      const cplx aq = cmul(a, {Q[re], Q[im]});
      X[re] += ap.re;
      X[im] += ap.im;
      const cplx r = {R[re] - aq.re, R[im] - aq.im};
      R[re] = r.re;
      R[im] = r.im;
      const cplx d = h == 0 ? diag_top(z, dS[e], dA[e]) : diag_bot(z, dS[e], dA[e]);
      const cplx u = cdiv(r, d);
      U[re] = u.re;
      U[im] = u.im;
    }
  }
}

// p = u + beta p
__global__ void cf_direction_kernel(long N, int nsys, const double* __restrict__ beta, const double* __restrict__ U,
                                    double* __restrict__ P) {
  CF_LOOP(idx, (long)nsys * N) {
    const long s = idx / N, e = idx % N;
    const cplx bt = {beta[2 * s], beta[2 * s + 1]};
    const long b = 4 * s * N + e;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long re = b + h * N, im = b + 2 * N + h * N;
      const cplx bp = cmul(bt, {P[re], P[im]});
      P[re] = U[re] + bp.re;
      P[im] = U[im] + bp.im;
    }
  }
}

// V: X_j = sum_q Re(w_q x_{q,j}) top rows, Y_j = the same over the bottom rows,
// w_q = r e^{i theta_q} / n
__global__ void cf_combine_kernel(long N, int k, int nq, const double* __restrict__ zw, const double* __restrict__ X,
                                  double* __restrict__ V) {
  CF_LOOP(idx, (long)k * N) {
    const long j = idx / N, e = idx % N;
    double sx = 0.0, sy = 0.0;
    for (int q = 0; q < nq; ++q) {
      const double wr = zw[4 * q + 2], wi = zw[4 * q + 3];
      const long b = 4 * ((long)q * k + j) * N + e;
      sx += wr * X[b] - wi * X[b + 2 * N];
      sy += wr * X[b + N] - wi * X[b + 3 * N];
    }
    V[j * N + e] = sx;
    V[(k + j) * N + e] = sy;
  }
}

}  // namespace

template <typename T>
T* ContourFilter::get(size_t n, const char* what) {
  T* p = c_.arena.alloc<T>(n, what);
  owned_.push_back(p);
  return p;
}

ContourFilter::ContourFilter(Context& c, int kblock, int nodes_max, int chunk, hipStream_t s)
    : c_(c), s_(s), N_(c.N), kblock_(kblock), nodes_max_(nodes_max), chunk_(chunk) {
  if (kblock < 1 || nodes_max < 1 || chunk < 2 * kblock) throw InvalidArg("contour filter: bad dimensions");
  const size_t rows = (size_t)4 * nodes_max * kblock;
  const size_t n = rows * N_;
  X_ = get<double>(n, "contour x");
  R_ = get<double>(n, "contour r");
  Z_ = get<double>(n, "contour u");
  P_ = get<double>(n, "contour p");
  Q_ = get<double>(n, "contour q");
  AP_ = get<double>(n, "contour Ap");
  BP_ = get<double>(n, "contour Bp");
  SP_ = get<double>(n, "contour Sp");
  const size_t ns = (size_t)nodes_max * kblock;
  rho_ = get<double>(2 * ns, "contour rho");
  rho2_ = get<double>(2 * ns, "contour rho'");
  sig_ = get<double>(2 * ns, "contour sigma");
  alpha_ = get<double>(2 * ns, "contour alpha");
  beta_ = get<double>(2 * ns, "contour beta");
  rn2_ = get<double>(ns, "contour |r|^2");
  bn2_ = get<double>(ns, "contour |b|^2");
  zw_ = get<double>((size_t)4 * nodes_max, "contour nodes");
  done_ = get<int>(ns, "contour done");
}

ContourFilter::~ContourFilter() {
  for (void* p : owned_) c_.arena.free(p);
}

size_t ContourFilter::bytes(long N, int kblock, int nodes_max) {
  auto r = [](size_t b) { return ((b + 255) / 256) * 256; };
  const size_t D = sizeof(double);
  const size_t ns = (size_t)nodes_max * kblock;
  return 8 * r(4 * ns * N * D) + 5 * r(2 * ns * D) + 2 * r(ns * D) + r(4 * (size_t)nodes_max * D) +
         r(ns * sizeof(int));
}

void ContourFilter::multiply(int rows, const double* X, const ProductFn& prod) {
  for (int r0 = 0; r0 < rows; r0 += chunk_) {
    const int kc = std::min(chunk_, rows - r0);
    const size_t off = (size_t)r0 * N_;
    prod(kc, X + off, AP_ + off, BP_ + off, SP_ + off);
    products_ += kc;
  }
}

int ContourFilter::apply(const ContourParams& p, int k, double* V, const ProductFn& prod, double* worst) {
  if (k < 1 || k > kblock_) throw InvalidArg("contour filter: block size out of range");
  if (p.nodes < 1 || p.nodes > nodes_max_) throw InvalidArg("contour filter: node count out of range");
  if (!(p.radius > 0.0) || !(p.tol > 0.0) || p.maxit < 1) throw InvalidArg("contour filter: bad contour");
  const int nq = p.nodes;
  const int nsys = nq * k;
  const long N = N_;
  // nodes z_q = c + r e^{i theta_q} and weights r e^{i theta_q} / n on the upper half circle
  std::vector<double> zw((size_t)4 * nq);
  for (int q = 0; q < nq; ++q) {
    const double th = 3.14159265358979323846 * (2.0 * q + 1.0) / (2.0 * nq);
    zw[4 * q] = p.center + p.radius * std::cos(th);
    zw[4 * q + 1] = p.radius * std::sin(th);
    zw[4 * q + 2] = p.radius * std::cos(th) / nq;
    zw[4 * q + 3] = p.radius * std::sin(th) / nq;
  }
  PPW_HIP(hipMemcpyAsync(zw_, zw.data(), sizeof(double) * zw.size(), hipMemcpyHostToDevice, s_));
  PPW_HIP(hipMemsetAsync(done_, 0, sizeof(int) * nsys, s_));
  // right-hand sides Sigma [X_j; Y_j]: S products of the block
  multiply(2 * k, V, prod);
  cf_init_kernel<<<grid_of((long)nsys * N), kT, 0, s_>>>(N, k, nq, zw_, c_.dA, c_.dS, SP_, X_, R_, Z_, P_);
  PPW_LAUNCH_CHECK();
  cf_dot_kernel<<<nsys, kT, 0, s_>>>(N, R_, Z_, rho_, bn2_);
  PPW_LAUNCH_CHECK();
  std::vector<double> bn2(nsys), rn2(nsys);
  PPW_HIP(hipMemcpyAsync(bn2.data(), bn2_, sizeof(double) * nsys, hipMemcpyDeviceToHost, s_));
  PPW_HIP(hipStreamSynchronize(s_));
  std::vector<int> done(nsys, 0);
  for (int s = 0; s < nsys; ++s) done[s] = bn2[s] == 0.0 ? 1 : 0;
  PPW_HIP(hipMemcpyAsync(done_, done.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, s_));
  const double tol2 = p.tol * p.tol;
  int it = 0;
  double wr = 0.0;
  for (it = 1; it <= p.maxit; ++it) {
    multiply(4 * nsys, P_, prod);
    cf_apply_kernel<<<grid_of((long)nsys * N), kT, 0, s_>>>(N, k, nsys, zw_, AP_, BP_, SP_, Q_);
    PPW_LAUNCH_CHECK();
    cf_dot_kernel<<<nsys, kT, 0, s_>>>(N, P_, Q_, sig_, nullptr);
    cf_alpha_kernel<<<1, kT, 0, s_>>>(nsys, rho_, sig_, done_, alpha_);
    cf_update_kernel<<<grid_of((long)nsys * N), kT, 0, s_>>>(N, k, nsys, zw_, alpha_, c_.dA, c_.dS, P_, Q_, X_, R_,
                                                              Z_);
    cf_dot_kernel<<<nsys, kT, 0, s_>>>(N, R_, Z_, rho2_, rn2_);
    PPW_LAUNCH_CHECK();
    PPW_HIP(hipMemcpyAsync(rn2.data(), rn2_, sizeof(double) * nsys, hipMemcpyDeviceToHost, s_));
    PPW_HIP(hipStreamSynchronize(s_));
    int left = 0;
    bool changed = false;
    wr = 0.0;
    for (int s = 0; s < nsys; ++s) {
      if (!std::isfinite(rn2[s])) throw Unstable("contour solve diverged");
      const double rel = bn2[s] > 0.0 ? std::sqrt(rn2[s] / bn2[s]) : 0.0;
      wr = std::max(wr, rel);
      if (!done[s] && rn2[s] <= tol2 * bn2[s]) {
        done[s] = 1;
        changed = true;
      }
      left += done[s] ? 0 : 1;
    }
    if (left == 0) break;
    if (changed) PPW_HIP(hipMemcpyAsync(done_, done.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, s_));
    cf_beta_kernel<<<1, kT, 0, s_>>>(nsys, rho_, rho2_, done_, beta_);
    cf_direction_kernel<<<grid_of((long)nsys * N), kT, 0, s_>>>(N, nsys, beta_, Z_, P_);
    PPW_LAUNCH_CHECK();
  }
  it = std::min(it, p.maxit);
  cf_combine_kernel<<<grid_of((long)k * N), kT, 0, s_>>>(N, k, nq, zw_, X_, V);
  PPW_LAUNCH_CHECK();
  // the host vectors above were sources of asynchronous copies
  PPW_HIP(hipStreamSynchronize(s_));
  if (worst) *worst = wr;
  return it;
}

}  // namespace ppw
