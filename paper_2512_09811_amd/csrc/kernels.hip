// Bandwidth-bound kernels: layout permutations, amplitude-strip formation,
// diagonals, product assembly and vector reductions.  All loops are grid-stride
// with 64-bit indices; reductions use wavefront shuffles in a fixed order so every
// result is bitwise reproducible.
#include "kernels.h"

#include <algorithm>

namespace ppw {
namespace {

constexpr int kBlock = 256;

inline int grid_for(long n, int block = kBlock) {
  long g = (n + block - 1) / block;
  return (int)std::max<long>(1, std::min<long>(g, 65536));
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// block-wide sum (blockDim.x == 256), result valid in thread 0
__device__ double block_sum(double v) {
  __shared__ double part[kBlock / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) s += part[w];
  __syncthreads();
  return s;
}

__global__ void permute3_kernel(const double* __restrict__ in, double* __restrict__ out, int d0, int d1, int d2,
                                int p0, int p1, int p2) {
  const int dims[3] = {d0, d1, d2};
  const int o0 = dims[p0], o1 = dims[p1], o2 = dims[p2];
  const long n = (long)d0 * d1 * d2;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    // idx enumerates the OUTPUT in row-major order (coalesced writes)
    const int c2 = (int)(idx % o2);
    const long r = idx / o2;
    const int c1 = (int)(r % o1);
    const int c0 = (int)(r / o1);
    int ii[3];
    ii[p0] = c0;
    ii[p1] = c1;
    ii[p2] = c2;
    out[idx] = in[((long)ii[0] * d1 + ii[1]) * d2 + ii[2]];
  }
}

template <typename T>
__global__ void tau_strip_kernel(const T* __restrict__ S, int o, int v, int k0, int ib, const double* __restrict__ eo,
                                 const double* __restrict__ ev, T* __restrict__ tau, long ldt, double* __restrict__ t,
                                 double* __restrict__ tEv, double* __restrict__ tEo, double* __restrict__ partial) {
  // block: one (k_local, l) pair and a 32x32 (x, y) tile; 256 threads, 4 elements each
  __shared__ T T1[32][33];
  __shared__ T T2[32][33];
  const int nt = (v + 31) / 32;
  const int tile = blockIdx.x;
  const int tx = tile % nt, ty = tile / nt;   // x tile, y tile
  const int kl = blockIdx.y;                  // (k_local, l) pair
  const int kloc = kl / o, l = kl % o;
  const int k = k0 + kloc;
  const long N = (long)o * v;
  const int x0 = tx * 32, y0 = ty * 32;
  const int tid = threadIdx.x;
  // T1[x][y] = S[(k, x0+x)][(l, y0+y)],  T2[y][x] = S[(k, y0+y)][(l, x0+x)]
  for (int e = tid; e < 1024; e += 256) {
    const int r = e / 32, c = e % 32;
    const int x = x0 + r, y = y0 + c;
    T a = T(0), b = T(0);
    if (x < v && y < v) a = S[((long)kloc * v + x) * N + (long)l * v + y];
    const int yy = y0 + r, xx = x0 + c;
    if (yy < v && xx < v) b = S[((long)kloc * v + yy) * N + (long)l * v + xx];
    T1[r][c] = a;
    T2[r][c] = b;
  }
  __syncthreads();
  double acc = 0.0;
  const double ekl = eo[k] + eo[l];
  for (int e = tid; e < 1024; e += 256) {
    const int r = e / 32, c = e % 32;
    const int x = x0 + r, y = y0 + c;
    if (x < v && y < v) {
      const double sxy = (double)T1[r][c];
      const double syx = (double)T2[c][r];
      const double D = ekl - ev[x] - ev[y];
      const double tt = sxy / D;
      const double tu = (2.0 * sxy - syx) / D;
      const long idx = ((long)kloc * v + x) * N + (long)l * v + y;
      if (tau) tau[((long)kloc * v + x) * ldt + (long)l * v + y] = (T)tu;
      if (t) t[idx] = tt;
      if (tEv) tEv[idx] = tt * (ekl - ev[y]);
      if (tEo) tEo[idx] = tt * (eo[k] - ev[x] - ev[y]);
      acc += tu * sxy;
    }
  }
  if (partial) {
    const double s = block_sum(acc);
    if (tid == 0) partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void sum_reduce_kernel(const double* __restrict__ x, long n, double* __restrict__ out) {
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) acc += x[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) *out = s;
}

__global__ void diag_integrals_kernel(const double* __restrict__ Bov, const double* __restrict__ Boo,
                                      const double* __restrict__ Bvv, int o, int v, int naux,
                                      double* __restrict__ coul, double* __restrict__ exch) {
  const long N = (long)o * v;
  for (long ia = blockIdx.x * (long)blockDim.x + threadIdx.x; ia < N; ia += (long)gridDim.x * blockDim.x) {
    const int i = (int)(ia / v), a = (int)(ia % v);
    double c = 0.0, x = 0.0;
    for (int P = 0; P < naux; ++P) {
      const double b = Bov[(long)P * N + ia];
      c += b * b;
      x += Boo[((long)P * o + i) * o + i] * Bvv[((long)P * v + a) * v + a];
    }
    coul[ia] = c;
    exch[ia] = x;
  }
}

__global__ void diag_assemble_kernel(int o, int v, int order, const double* __restrict__ eo,
                                     const double* __restrict__ ev, const double* __restrict__ coul,
                                     const double* __restrict__ exch, const double* __restrict__ Gv,
                                     const double* __restrict__ Ev, const double* __restrict__ Go,
                                     const double* __restrict__ Eo, double* __restrict__ dA, double* __restrict__ dB,
                                     double* __restrict__ dS) {
  const long N = (long)o * v;
  for (long ia = blockIdx.x * (long)blockDim.x + threadIdx.x; ia < N; ia += (long)gridDim.x * blockDim.x) {
    const int i = (int)(ia / v), a = (int)(ia % v);
    double A = ev[a] - eo[i], B = 0.0, S = 1.0;
    if (order >= 1) {
      A += 2.0 * coul[ia] - exch[ia];
      B = coul[ia];
    }
    if (order >= 2) {
      const double gv = Gv[(long)a * v + a], ee = Ev[(long)a * v + a];
      const double go = Go[(long)i * o + i], eoo = Eo[(long)i * o + i];
      A += -(ee - eo[i] * gv) - (ev[a] * go + eoo);
      S -= go + gv;
    }
    dA[ia] = A;
    dB[ia] = B;
    dS[ia] = S;
  }
}

__global__ void sigma_assemble_kernel(int o, int v, int k, int order, const double* __restrict__ eo,
                                      const double* __restrict__ ev, const double* __restrict__ V,
                                      const double* __restrict__ J, const double* __restrict__ P1,
                                      const double* __restrict__ P2, const double* __restrict__ P3,
                                      const double* __restrict__ P4, double* __restrict__ AV, double* __restrict__ BV,
                                      double* __restrict__ SV) {
  const long N = (long)o * v;
  const long n = N * k;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    const long ia = idx % N;
    const int i = (int)(ia / v), a = (int)(ia % v);
    const double x = V[idx];
    double av = (ev[a] - eo[i]) * x;
    double bv = 0.0;
    double sv = x;
    if (order >= 1) {
      const double j2 = 2.0 * J[idx];
      av += j2 + AV[idx];
      bv = j2 + BV[idx];
    }
    if (order >= 2) {
      av += -P2[idx] + eo[i] * P1[idx] - ev[a] * P3[idx] - P4[idx];
      sv -= P3[idx] + P1[idx];
    }
    AV[idx] = av;
    BV[idx] = bv;
    if (SV) SV[idx] = sv;
  }
}

__global__ void ring_operand_kernel(const double* __restrict__ Bov, const double* __restrict__ Lam, int o, int v,
                                    int naux, double* __restrict__ R) {
  // output R[j][s][P][a] (s in {0,1} when Lam != null) enumerated row-major
  const int ns = Lam ? 2 : 1;
  const long n = (long)o * ns * naux * v;
  const long N = (long)o * v;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    const int a = (int)(idx % v);
    long r = idx / v;
    const int P = (int)(r % naux);
    r /= naux;
    const int s = (int)(r % ns);
    const int j = (int)(r / ns);
    const long src = (long)P * N + (long)j * v + a;
    double val = Bov[src];
    if (Lam && s == 0) val += Lam[src];
    R[idx] = val;
  }
}

__global__ void axpby_kernel(long n, double alpha, const double* __restrict__ x, double beta, double* __restrict__ y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = alpha * x[i] + (beta == 0.0 ? 0.0 : beta * y[i]);
}

__global__ void to_f32_kernel(long n, const double* __restrict__ x, float* __restrict__ y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// one block per bin: pairs with eps_a - eps_i in [lo, hi); sums in a fixed order
__global__ void dos_kernel(int o, int v, const double* __restrict__ eo, const double* __restrict__ ev,
                           const double* __restrict__ dip, const double* __restrict__ edges, double* __restrict__ out) {
  const int b = blockIdx.x;
  const double lo = edges[b], hi = edges[b + 1];
  const long N = (long)o * v;
  double cnt = 0.0, m2 = 0.0;
  for (long ia = threadIdx.x; ia < N; ia += blockDim.x) {
    const int i = (int)(ia / v), a = (int)(ia % v);
    const double d = ev[a] - eo[i];
    if (d >= lo && d < hi) {
      cnt += 1.0;
      if (dip) m2 += dip[ia] * dip[ia] + dip[N + ia] * dip[N + ia] + dip[2 * N + ia] * dip[2 * N + ia];
    }
  }
  cnt = block_sum(cnt);
  m2 = block_sum(m2);
  if (threadIdx.x == 0) {
    out[2 * b] = cnt;
    out[2 * b + 1] = m2;
  }
}

__global__ void response_kernel(int n, const double* __restrict__ e, const double* __restrict__ f, int ng,
                                const double* __restrict__ om, double eta, double* __restrict__ re,
                                double* __restrict__ im, double* __restrict__ lor) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const double w = om[g];
  double sr = 0.0, si = 0.0, sl = 0.0;
  const double eta2 = eta * eta;
  for (int k = 0; k < n; ++k) {
    const double c = f[k] / (2.0 * e[k]);
    const double dm = w - e[k], dp = w + e[k];
    const double qm = 1.0 / (dm * dm + eta2), qp = 1.0 / (dp * dp + eta2);
    // 1 / (d + i eta) = (d - i eta) / (d^2 + eta^2)
    sr += c * (dm * qm - dp * qp);
    si += c * (-eta * qm + eta * qp);
    sl += f[k] * qm;
  }
  if (re) re[g] = sr;
  if (im) im[g] = si;
  if (lor) lor[g] = sl * eta * 0.31830988618379067154;  // eta / pi
}

__global__ void fill_zero_kernel(long n, double* __restrict__ y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = 0.0;
}

__global__ void to_f32_rows_kernel(long rows, long cols, const double* __restrict__ x, long ldx,
                                   float* __restrict__ y, long ldy) {
  const long n = rows * ldy;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    const long r = idx / ldy, c = idx % ldy;
    y[idx] = c < cols ? (float)x[r * ldx + c] : 0.0f;
  }
}

// 32 x 32 tiles through LDS: reads along x's rows, writes along y's rows.
__global__ void transpose_to_f32_kernel(long rows, long cols, const double* __restrict__ x, float* __restrict__ y,
                                        long ldy) {
  __shared__ float tile[32][33];
  const long r0 = (long)blockIdx.y * 32, c0 = (long)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows of 32
  for (int i = ty; i < 32; i += 8) {
    const long r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? (float)x[r * cols + c] : 0.0f;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const long c = c0 + i, r = r0 + tx;
    if (c < cols && r < ldy) y[c * ldy + r] = tile[tx][i];
  }
}

__global__ void to_f64_kernel(long n, const float* __restrict__ x, double* __restrict__ y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

// one block per column; fixed reduction order
__global__ void column_dots_kernel(const double* __restrict__ x, const double* __restrict__ y, long n,
                                   double* __restrict__ out) {
  const int c = blockIdx.x;
  const double* xc = x + (long)c * n;
  const double* yc = y + (long)c * n;
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) acc += xc[i] * yc[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) out[c] = s;
}

__global__ void combine_pairs_kernel(long N, int m, const double* __restrict__ AV, const double* __restrict__ BV,
                                     const double* __restrict__ SV, int metric, double* __restrict__ out) {
  const long n = 2 * N * m;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    const long r = idx % N;
    const long qh = idx / N;
    const int q = (int)(qh / 2), h = (int)(qh % 2);
    const long a = (long)q * N + r, b = (long)(m + q) * N + r;
    double val;
    if (metric)
      val = h == 0 ? SV[a] : -SV[b];
    else
      val = h == 0 ? AV[a] + BV[b] : BV[a] + AV[b];
    out[idx] = val;
  }
}

}  // namespace

void combine_pairs(long N, int m, const double* AV, const double* BV, const double* SV, bool metric, double* out,
                   hipStream_t s) {
  const long n = 2 * N * m;
  combine_pairs_kernel<<<grid_for(n), kBlock, 0, s>>>(N, m, AV, BV, SV, metric ? 1 : 0, out);
  PPW_LAUNCH_CHECK();
}

void permute3(const double* in, double* out, int d0, int d1, int d2, const int perm[3], hipStream_t s) {
  const long n = (long)d0 * d1 * d2;
  permute3_kernel<<<grid_for(n), kBlock, 0, s>>>(in, out, d0, d1, d2, perm[0], perm[1], perm[2]);
  PPW_LAUNCH_CHECK();
}

long tau_blocks(int o, int v, int ib) {
  const long nt = (v + 31) / 32;
  return nt * nt * (long)ib * o;
}

void tau_strip(const double* S, int o, int v, int k0, int ib, const double* eps_o, const double* eps_v, double* tau,
               double* t, double* tEv, double* tEo, double* partial, hipStream_t s) {
  const int nt = (v + 31) / 32;
  dim3 grid(nt * nt, ib * o);
  tau_strip_kernel<double><<<grid, 256, 0, s>>>(S, o, v, k0, ib, eps_o, eps_v, tau, (long)o * v, t, tEv, tEo,
                                                 partial);
  PPW_LAUNCH_CHECK();
}

void tau_strip_f32(const float* S, int o, int v, int k0, int ib, const double* eps_o, const double* eps_v, float* tau,
                   long ld, hipStream_t s) {
  const int nt = (v + 31) / 32;
  dim3 grid(nt * nt, ib * o);
  tau_strip_kernel<float><<<grid, 256, 0, s>>>(S, o, v, k0, ib, eps_o, eps_v, tau, ld, nullptr, nullptr, nullptr,
                                                nullptr);
  PPW_LAUNCH_CHECK();
}

void sum_reduce(const double* x, long n, double* out, hipStream_t s) {
  sum_reduce_kernel<<<1, kBlock, 0, s>>>(x, n, out);
  PPW_LAUNCH_CHECK();
}

void diag_integrals(const double* Bov, const double* Boo, const double* Bvv, int o, int v, int naux, double* coul,
                    double* exch, hipStream_t s) {
  diag_integrals_kernel<<<grid_for((long)o * v), kBlock, 0, s>>>(Bov, Boo, Bvv, o, v, naux, coul, exch);
  PPW_LAUNCH_CHECK();
}

void diag_assemble(int o, int v, int order, const double* eps_o, const double* eps_v, const double* coul,
                   const double* exch, const double* Gv, const double* Ev, const double* Go, const double* Eo,
                   double* dA, double* dB, double* dS, hipStream_t s) {
  diag_assemble_kernel<<<grid_for((long)o * v), kBlock, 0, s>>>(o, v, order, eps_o, eps_v, coul, exch, Gv, Ev, Go,
                                                                 Eo, dA, dB, dS);
  PPW_LAUNCH_CHECK();
}

void sigma_assemble(int o, int v, int k, int order, const double* eps_o, const double* eps_v, const double* V,
                    const double* J, const double* P1, const double* P2, const double* P3, const double* P4,
                    double* AV, double* BV, double* SV, hipStream_t s) {
  const long n = (long)o * v * k;
  sigma_assemble_kernel<<<grid_for(n), kBlock, 0, s>>>(o, v, k, order, eps_o, eps_v, V, J, P1, P2, P3, P4, AV, BV,
                                                        SV);
  PPW_LAUNCH_CHECK();
}

void build_ring_operand(const double* Bov, const double* Lam, int o, int v, int naux, double* R, hipStream_t s) {
  const long n = (long)o * (Lam ? 2 : 1) * naux * v;
  ring_operand_kernel<<<grid_for(n), kBlock, 0, s>>>(Bov, Lam, o, v, naux, R);
  PPW_LAUNCH_CHECK();
}

void axpby(long n, double alpha, const double* x, double beta, double* y, hipStream_t s) {
  axpby_kernel<<<grid_for(n), kBlock, 0, s>>>(n, alpha, x, beta, y);
  PPW_LAUNCH_CHECK();
}

void to_f32(long n, const double* x, float* y, hipStream_t s) {
  to_f32_kernel<<<grid_for(n), kBlock, 0, s>>>(n, x, y);
  PPW_LAUNCH_CHECK();
}

void response_on_grid(int n, const double* e, const double* f, int n_omega, const double* omega, double eta,
                      double* re, double* im, double* lor, hipStream_t s) {
  if (n_omega <= 0) return;
  response_kernel<<<(n_omega + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, e, f, n_omega, omega, eta, re, im, lor);
  PPW_LAUNCH_CHECK();
}

void fill_zero(long n, double* y, hipStream_t s) {
  if (n <= 0) return;
  fill_zero_kernel<<<grid_for(n), kBlock, 0, s>>>(n, y);
  PPW_LAUNCH_CHECK();
}

void to_f32_rows(long rows, long cols, const double* x, long ldx, float* y, long ldy, hipStream_t s) {
  to_f32_rows_kernel<<<grid_for(rows * ldy), kBlock, 0, s>>>(rows, cols, x, ldx, y, ldy);
  PPW_LAUNCH_CHECK();
}

void transpose_to_f32(long rows, long cols, const double* x, float* y, long ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  // padded rows of y (r >= rows up to ldy) are covered by the tiles of the last block row
  const long brows = (std::max(rows, ldy) + 31) / 32, bcols = (cols + 31) / 32;
  if (brows > 65535) throw InvalidArg("transpose_to_f32: too many rows");
  transpose_to_f32_kernel<<<dim3((unsigned)bcols, (unsigned)brows), kBlock, 0, s>>>(rows, cols, x, y, ldy);
  PPW_LAUNCH_CHECK();
}

void exciton_dos(int o, int v, const double* eo, const double* ev, const double* dip, const double* edges,
                 int n_bins, double* out, hipStream_t s) {
  dos_kernel<<<n_bins, kBlock, 0, s>>>(o, v, eo, ev, dip, edges, out);
  PPW_LAUNCH_CHECK();
}

void to_f64(long n, const float* x, double* y, hipStream_t s) {
  to_f64_kernel<<<grid_for(n), kBlock, 0, s>>>(n, x, y);
  PPW_LAUNCH_CHECK();
}

void column_dots(const double* x, const double* y, long n, int k, double* out, hipStream_t s) {
  if (k <= 0) return;
  column_dots_kernel<<<k, kBlock, 0, s>>>(x, y, n, out);
  PPW_LAUNCH_CHECK();
}

}  // namespace ppw
