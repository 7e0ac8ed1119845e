// Setup of a system and the matrix-free product of the response matrix.
//
// Working equations (closed-shell singlet, density-fitted; index ia = i*v + a),
// for a block V of k particle-hole vectors:
//
//   first order   A V = Delta V + 2 J(V) - K_A(V),   B V = 2 J(V) - K_B(V)
//                 J(V)_ia  = sum_P B_P,ia sum_jb B_P,jb V_jb
//                 K_A(V)   = sum_P B^oo_P V B^vv_P
//                 K_B(V)   = sum_P B^ov_P V^T B^ov_P
//   second order  S V     += -Go V - V Gv
//                 A V     += -V Ev + e_i (V Gv) - e_a (Go V) - Eo V
//                 B V     += sum_P (H_P B^vv_P - B^oo_P H_P)
//                            - sum_P (B^ov_P V^T Lam_P + Lam_P V^T B^ov_P)
//                 G_P = V B^vv_P - B^oo_P V,  H_P,ic = sum_jd tau_ij^cd G_P,jd
//
// with tau_ij^ab = 2 t_ij^ab - t_ij^ba, t_ij^ab = (ia|jb)/(e_i + e_j - e_a - e_b),
// Gv/Ev/Go/Eo the (energy-weighted) MP2 densities and Lam_P,ia = sum_kc tau_ik^ac B_P,kc.
// These are the closed forms of the second-order expectation values of the
// second-order section (metric, A and B over the MP2 ground state), written
// through the DF factors so that no four-index quantity except amplitude strips
// tau_i (v x N per occupied i) is ever formed.  The dominant contraction is
// H = tau G (o^2 v^2 naux k multiply-adds); with stored amplitudes it is one
// N x N x (naux k) GEMM, otherwise one GEMM per strip batch after the strip is
// rebuilt from B^ov (K = naux) and the denominators.
#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "context.h"
#include "kernels.h"

namespace ppw {

Context::~Context() {
  arena.release();
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

namespace {

GemmDesc gd(int M, int N, int K, int transA, long lda, int transB, long ldb, long ldc) {
  GemmDesc d;
  d.M = M;
  d.N = N;
  d.K = K;
  d.transA = transA;
  d.lda = lda;
  d.transB = transB;
  d.ldb = ldb;
  d.ldc = ldc;
  return d;
}

void copy_in(double* dst, const double* src, size_t n, bool dev, hipStream_t s) {
  PPW_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}

void ensure_ws(Context& c, size_t bytes) {
  if (bytes <= c.ws_bytes) return;
  if (c.ws.ptr) c.arena.free(c.ws.ptr);
  c.ws.ptr = c.arena.alloc<char>(bytes, "split-K workspace");
  c.ws.bytes = bytes;
  c.ws_bytes = bytes;
}

// rows per amplitude strip batch that fit 'bytes' with 'arrays' strip-sized arrays
int strip_rows_for(const Context& c, size_t bytes, int arrays) {
  const size_t per_row = (size_t)c.v * c.N * sizeof(double) * arrays;
  int ib = (int)std::max<size_t>(1, bytes / std::max<size_t>(per_row, 1));
  return std::min(ib, c.o);
}

}  // namespace

// Whether the amplitudes the given precision's products read are stored (else they are
// rebuilt in strips in every pass).
static bool amplitudes_stored(const Context& c, int prec) {
  if (prec == 1) return c.split_bf16 ? c.tau_sbf != nullptr : c.tau32 != nullptr;
  return c.tau != nullptr;
}

// Algorithmic flops of the part of a pass that does not depend on the amplitude strips
// (pre) and of the strips of 'rows' occupied rows.
static void pass_flops(const Context& c, int order, int k, int prec, int rows, double* pre, double* strips) {
  *pre = *strips = 0.0;
  if (order <= 0) return;
  const double o = c.o, v = c.v, X = c.naux, N = (double)c.N, K = k;
  double f = 0.0;
  f += 2.0 * X * N * K * 2.0;                  // J (two GEMMs)
  f += 2.0 * K * X * o * v * v;                // V B^vv_P for all P
  f += 2.0 * K * X * o * o * v;                // sum_P B^oo_P (.)   (K_A)
  const double ns = order >= 2 ? 2.0 : 1.0;
  f += 2.0 * K * o * v * ns * X * o;           // V^T [B^ov; Lam]
  f += 2.0 * K * o * ns * X * o * v;           // ring / K_B output
  double g = 0.0;
  if (order >= 2) {
    f += 2.0 * K * X * o * o * v;              // - B^oo_P V   (G)
    f += 2.0 * K * o * v * v * 2.0;            // V Gv, V Ev
    f += 2.0 * K * o * o * v * 2.0;            // Go V, Eo V
    g += 2.0 * N * N * K * X;                  // H = tau G    (dominant)
    if (!amplitudes_stored(c, prec)) g += 2.0 * N * N * X;  // (ia|jb) of the rebuilt strips
    g += 2.0 * K * X * o * v * v;              // H B^vv
    g += 2.0 * K * X * o * o * v;              // B^oo H
  }
  *pre = f;
  // stored amplitudes: the whole contraction runs with the prologue
  if (order >= 2 && amplitudes_stored(c, prec))
    *pre += g;
  else
    *strips = g * rows / o;
}

double sigma_flops(const Context& c, int order, int k, int prec) {
  double pre, strips;
  pass_flops(c, order, k, prec, c.o, &pre, &strips);
  return pre + strips;
}

Context* setup_context(const SetupParams& p) {
  if (p.o < 1 || p.v < 1 || p.naux < 1) throw InvalidArg("n_occ, n_vir and n_aux must be positive");
  if (p.order < 0 || p.order > 2) throw InvalidArg("order must be 0, 1 or 2");
  if (!p.eps || !p.Boo || !p.Bov || !p.Bvv) throw InvalidArg("eps, B_oo, B_ov and B_vv are required");
  if ((long)p.o * p.v > 2147483647L / 2) throw InvalidArg("particle-hole dimension too large");
  auto* c = new Context();
  try {
    c->o = p.o;
    c->v = p.v;
    c->naux = p.naux;
    c->order = p.order;
    c->split_bf16 = p.split_bf16 && p.want_f32;
    c->N = (long)p.o * p.v;
    c->N8 = padded_stride(c->N);
    c->X8 = (p.naux + 7) / 8 * 8;
    c->device = p.device;
    PPW_HIP(hipSetDevice(p.device));
    if (p.stream) {
      c->stream = p.stream;
    } else {
      PPW_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    size_t freeb = 0, totalb = 0;
    PPW_HIP(hipMemGetInfo(&freeb, &totalb));
    c->arena.set_budget(p.budget ? p.budget : (size_t)(0.9 * (double)freeb));
    hipStream_t s = c->stream;
    const int o = p.o, v = p.v, X = p.naux;
    const long N = c->N;

    c->eps_o = c->arena.alloc<double>(o, "eps_o");
    c->eps_v = c->arena.alloc<double>(v, "eps_v");
    c->Boo = c->arena.alloc<double>((size_t)X * o * o, "B_oo");
    c->Bvv = c->arena.alloc<double>((size_t)X * v * v, "B_vv");
    c->ns = p.order >= 2 ? 2 : 1;
    c->BovLam = c->arena.alloc<double>((size_t)c->ns * X * N, "B_ov");
    c->Bov = c->BovLam;
    if (p.order >= 2) c->Lam = c->BovLam + (size_t)X * N;
    copy_in(c->eps_o, p.eps, o, p.device_ptrs, s);
    copy_in(c->eps_v, p.eps + o, v, p.device_ptrs, s);
    copy_in(c->Boo, p.Boo, (size_t)X * o * o, p.device_ptrs, s);
    copy_in(c->Bov, p.Bov, (size_t)X * N, p.device_ptrs, s);
    copy_in(c->Bvv, p.Bvv, (size_t)X * v * v, p.device_ptrs, s);
    if (p.dip) {
      c->dip = c->arena.alloc<double>((size_t)3 * N, "dip");
      copy_in(c->dip, p.dip, (size_t)3 * N, p.device_ptrs, s);
    }
    // layouts
    c->Boo_t = c->arena.alloc<double>((size_t)o * o * X, "B_oo [i][j][P]");
    const int perm[3] = {1, 2, 0};
    permute3(c->Boo, c->Boo_t, X, o, o, perm, s);
    ensure_ws(*c, std::max<size_t>((size_t)64 << 20, (size_t)X * 1024 * sizeof(double)));

    double* coul = c->arena.alloc<double>(N, "diag tmp");
    double* exch = c->arena.alloc<double>(N, "diag tmp");
    diag_integrals(c->Bov, c->Boo, c->Bvv, o, v, X, coul, exch, s);
    c->dA = c->arena.alloc<double>(N, "diag A");
    c->dB = c->arena.alloc<double>(N, "diag B");
    c->dS = c->arena.alloc<double>(N, "diag S");

    if (p.order >= 2) {
      c->Gv = c->arena.alloc<double>((size_t)v * v, "Gv");
      c->Ev = c->arena.alloc<double>((size_t)v * v, "Ev");
      c->Go = c->arena.alloc<double>((size_t)o * o, "Go");
      c->Eo = c->arena.alloc<double>((size_t)o * o, "Eo");
      PPW_HIP(hipMemsetAsync(c->Gv, 0, sizeof(double) * v * v, s));
      PPW_HIP(hipMemsetAsync(c->Ev, 0, sizeof(double) * v * v, s));
      PPW_HIP(hipMemsetAsync(c->Go, 0, sizeof(double) * o * o, s));
      PPW_HIP(hipMemsetAsync(c->Eo, 0, sizeof(double) * o * o, s));
      // amplitudes: store them all when requested / when they fit comfortably
      const size_t tau_bytes = (size_t)N * N * sizeof(double);
      bool store = p.store_amplitudes == 1;
      if (p.store_amplitudes < 0)
        store = c->arena.used() + 6 * tau_bytes < c->arena.budget() / 2;
      if (store) c->tau = c->arena.alloc<double>((size_t)N * N, "amplitudes tau");
      // strip batch size for the setup (S, tau, t, tEv, tEo = 5 arrays)
      const size_t room = c->arena.budget() > c->arena.used() ? c->arena.budget() - c->arena.used() : 0;
      int ib = p.strip_rows > 0 ? std::min(p.strip_rows, o) : strip_rows_for(*c, room / 3, store ? 4 : 5);
      c->strip_rows = ib;
      const size_t strip = (size_t)ib * v * N;
      double* S = c->arena.alloc<double>(strip, "strip S");
      double* tauS = store ? nullptr : c->arena.alloc<double>(strip, "strip tau");
      double* t = c->arena.alloc<double>(strip, "strip t");
      double* tEv = c->arena.alloc<double>(strip, "strip tEv");
      double* tEo = c->arena.alloc<double>(strip, "strip tEo");
      const long nblk = tau_blocks(o, v, ib);
      double* partial = c->arena.alloc<double>((size_t)nblk * ((o + ib - 1) / ib), "energy partials");
      long pofs = 0;
      for (int k0 = 0; k0 < o; k0 += ib) {
        const int nb = std::min(ib, o - k0);
        double* tau_b = store ? c->tau + (size_t)k0 * v * N : tauS;
        // S[(k,x)][(l,y)] = sum_P B_P,kx B_P,ly
        GemmDesc d = gd(nb * v, (int)N, X, 1, N, 0, N, N);
        gemm_f64(d, 1.0, c->Bov + (size_t)k0 * v, c->Bov, 0.0, S, s, c->ws);
        tau_strip(S, o, v, k0, nb, c->eps_o, c->eps_v, tau_b, t, tEv, tEo, partial + pofs, s);
        pofs += tau_blocks(o, v, nb);
        // Gv[a][b] += sum_k sum_(l,y) tau[(k,a)][(l,y)] t[(k,b)][(l,y)]
        GemmDesc g = gd(v, v, (int)N, 0, N, 1, N, v);
        g.KB = nb;
        g.sAk = (long)v * N;
        g.sBk = (long)v * N;
        gemm_f64(g, 1.0, tau_b, t, 1.0, c->Gv, s, c->ws);
        gemm_f64(g, 1.0, tau_b, tEv, 1.0, c->Ev, s, c->ws);
        // Go[i][j] += sum_(k,x) sum_y tau[(k,x)][(i,y)] t[(k,x)][(j,y)]
        GemmDesc h = gd(o, o, v, 0, v, 1, v, o);
        h.KB = nb * v;
        h.sAk = N;
        h.sBk = N;
        gemm_f64(h, 1.0, tau_b, t, 1.0, c->Go, s, c->ws);
        gemm_f64(h, 1.0, tau_b, tEo, 1.0, c->Eo, s, c->ws);
        // Lam[P][(i,a)] = sum_(l,y) Bov[P][(l,y)] tau[(i,a)][(l,y)]   (i in batch)
        GemmDesc l = gd(X, nb * v, (int)N, 0, N, 1, N, N);
        gemm_f64(l, 1.0, c->Bov, tau_b, 0.0, c->Lam + (size_t)k0 * v, s, c->ws);
      }
      double* e2 = c->arena.alloc<double>(1, "emp2");
      sum_reduce(partial, pofs, e2, s);
      PPW_HIP(hipMemcpyAsync(&c->emp2, e2, sizeof(double), hipMemcpyDeviceToHost, s));
      PPW_HIP(hipStreamSynchronize(s));
      c->arena.free(partial);
      c->arena.free(tEo);
      c->arena.free(tEv);
      c->arena.free(t);
      if (tauS) c->arena.free(tauS);
      c->arena.free(S);
      c->arena.free(e2);
    }
    diag_assemble(o, v, p.order, c->eps_o, c->eps_v, coul, exch, c->Gv, c->Ev, c->Go, c->Eo, c->dA, c->dB, c->dS,
                  s);
    c->tda = p.tda;
    if (c->tda) PPW_HIP(hipMemsetAsync(c->dB, 0, sizeof(double) * N, s));
    if (c->dip && p.order >= 2) {
      // property vector over the MP2 ground state through second order: S mu, with
      // S V = V - Go V - V Gv (the metric), for the three dipole components
      c->dipS = c->arena.alloc<double>((size_t)3 * N, "dip S mu");
      PPW_HIP(hipMemcpyAsync(c->dipS, c->dip, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, s));
      GemmDesc g1 = gd(o, v, o, 0, o, 0, v, v);  // - Go mu_x
      g1.nb1 = 3;
      g1.sB1 = N;
      g1.sC1 = N;
      gemm_f64(g1, -1.0, c->Go, c->dip, 1.0, c->dipS, s, c->ws);
      GemmDesc g2 = gd(o, v, v, 0, v, 0, v, v);  // - mu_x Gv
      g2.nb1 = 3;
      g2.sA1 = N;
      g2.sC1 = N;
      gemm_f64(g2, -1.0, c->dip, c->Gv, 1.0, c->dipS, s, c->ws);
    } else {
      c->dipS = c->dip;
    }
    c->R = c->arena.alloc<double>((size_t)o * c->ns * X * v, "ring operand");
    build_ring_operand(c->Bov, c->Lam, o, v, X, c->R, s);
    if (p.want_f32 && p.order >= 1) {
      // FP32 copies of every operand of the reduced-precision product path
      auto cp32 = [&](const double* src, size_t n, const char* w) {
        float* d = c->arena.alloc<float>(n, w);
        to_f32((long)n, src, d, s);
        return d;
      };
      c->BovLam32 = cp32(c->BovLam, (size_t)c->ns * X * N, "B_ov fp32");
      c->Boo32 = cp32(c->Boo, (size_t)X * o * o, "B_oo fp32");
      c->Bvv32 = cp32(c->Bvv, (size_t)X * v * v, "B_vv fp32");
      c->Boo_t32 = cp32(c->Boo_t, (size_t)o * o * X, "B_oo [i][j][P] fp32");
      c->R32 = cp32(c->R, (size_t)o * c->ns * X * v, "ring operand fp32");
      if (p.order >= 2 && c->split_bf16) {
        // operands of the split-BF16 amplitude products, split once here: the stored
        // amplitudes, or B^ov transposed for the integrals of the rebuilt strips
        if (c->tau) {
          c->tau_sbf = c->arena.alloc<float>((size_t)N * c->N8, "amplitudes tau split-BF16");
          to_f32_rows(N, N, c->tau, N, c->tau_sbf, c->N8, s);
          split_sbf16(N * c->N8, c->tau_sbf, s);
        } else {
          c->BovT_sbf = c->arena.alloc<float>((size_t)N * c->X8, "B_ov transposed split-BF16");
          transpose_to_f32(X, N, c->Bov, c->BovT_sbf, c->X8, s);
          split_sbf16(N * c->X8, c->BovT_sbf, s);
        }
      }
      if (p.order >= 2) {
        if (c->tau && !c->split_bf16) c->tau32 = cp32(c->tau, (size_t)N * N, "amplitudes tau fp32");
        c->Gv32 = cp32(c->Gv, (size_t)v * v, "Gv fp32");
        c->Ev32 = cp32(c->Ev, (size_t)v * v, "Ev fp32");
        c->Go32 = cp32(c->Go, (size_t)o * o, "Go fp32");
        c->Eo32 = cp32(c->Eo, (size_t)o * o, "Eo fp32");
      }
    }
    PPW_HIP(hipStreamSynchronize(s));
    c->arena.free(exch);
    c->arena.free(coul);
    if (c->strip_rows == 0) c->strip_rows = o;
  } catch (...) {
    delete c;
    throw;
  }
  return c;
}

namespace {

template <typename T>
T* regrow(Context& c, T*& p, size_t n, const char* w) {
  if (p) c.arena.free(p);
  p = c.arena.alloc<T>(n, w);
  return p;
}

// FP64 buffers every product pass needs for the final (FP64) assembly
void grow_assembly(Context& c, int k) {
  if (k <= c.kcap_asm) return;
  regrow(c, c.w_J, (size_t)k * c.N, "ws J");
  regrow(c, c.w_P, (size_t)4 * k * c.N, "ws P");
  c.kcap_asm = k;
}

void grow_workspace(Context& c, int k) {
  grow_assembly(c, k);
  if (k <= c.kcap) return;
  const int o = c.o, v = c.v, X = c.naux;
  const long N = c.N;
  regrow(c, c.w_c, (size_t)X * k, "ws c");
  regrow(c, c.w_G, (size_t)k * X * N, "ws G");
  regrow(c, c.w_U, (size_t)k * o * c.ns * X * o, "ws U");
  if (c.order >= 2) {
    const int ib = c.tau ? o : c.strip_rows;
    regrow(c, c.w_H, (size_t)ib * v * k * X, "ws H");
    if (!c.tau) {
      regrow(c, c.w_S, (size_t)c.strip_rows * v * N, "ws strip S");
      regrow(c, c.w_tau, (size_t)c.strip_rows * v * N, "ws strip tau");
    }
  }
  c.kcap = k;
}

void grow_workspace32(Context& c, int k) {
  grow_assembly(c, k);
  if (k <= c.kcap32) return;
  const int o = c.o, v = c.v, X = c.naux;
  const long N = c.N;
  regrow(c, c.w32_V, (size_t)k * N, "ws32 V");
  regrow(c, c.w32_AV, (size_t)k * N, "ws32 AV");
  regrow(c, c.w32_BV, (size_t)k * N, "ws32 BV");
  regrow(c, c.w32_J, (size_t)k * N, "ws32 J");
  regrow(c, c.w32_P, (size_t)4 * k * N, "ws32 P");
  regrow(c, c.w32_c, (size_t)X * k, "ws32 c");
  // G rows (q,P) of N8 values; the padding past N stays zero (split-BF16 chunks)
  regrow(c, c.w32_G, (size_t)k * X * c.N8, "ws32 G");
  PPW_HIP(hipMemsetAsync(c.w32_G, 0, sizeof(float) * k * X * c.N8, c.stream));
  PPW_HIP(hipStreamSynchronize(c.stream));  // products may run on another stream
  regrow(c, c.w32_U, (size_t)k * o * c.ns * X * o, "ws32 U");
  if (c.order >= 2) {
    const bool stored = amplitudes_stored(c, 1);
    const int ib = stored ? o : c.strip_rows;
    regrow(c, c.w32_H, (size_t)ib * v * k * X, "ws32 H");
    if (!stored) {
      regrow(c, c.w32_S, (size_t)c.strip_rows * v * N, "ws32 strip S");
      regrow(c, c.w32_tau, (size_t)c.strip_rows * v * c.N8, "ws32 strip tau");
      PPW_HIP(hipMemsetAsync(c.w32_tau, 0, sizeof(float) * c.strip_rows * v * c.N8, c.stream));
      PPW_HIP(hipStreamSynchronize(c.stream));
    }
  }
  c.kcap32 = k;
}

template <typename T>
void gemm_t(const GemmDesc& d, T a, const T* A, const T* B, T b, T* C, hipStream_t s, Workspace ws);
template <>
void gemm_t<double>(const GemmDesc& d, double a, const double* A, const double* B, double b, double* C,
                    hipStream_t s, Workspace ws) {
  gemm_f64(d, a, A, B, b, C, s, ws);
}
template <>
void gemm_t<float>(const GemmDesc& d, float a, const float* A, const float* B, float b, float* C, hipStream_t s,
                   Workspace ws) {
  gemm_f32(d, a, A, B, b, C, s, ws);
}
// Split-BF16 amplitude contraction (FP32 operands only).
inline void gemm_sbf16_t(const GemmDesc& d, float a, const float* A, const float* B, float b, float* C,
                         hipStream_t s, bool amplitude) {
  gemm_sbf16(d, a, A, B, b, C, s, amplitude);
}
inline void gemm_sbf16_t(const GemmDesc&, double, const double*, const double*, double, double*, hipStream_t, bool) {
  throw InvalidArg("split-BF16 products take FP32 operands");
}

template <typename T>
void gemm_hhat_t(const GemmDesc& d, T a, const T* A, const T* B, T b, T* C, hipStream_t s, Workspace ws);
template <>
void gemm_hhat_t<double>(const GemmDesc& d, double a, const double* A, const double* B, double b, double* C,
                         hipStream_t s, Workspace ws) {
  gemm_f64_hhat(d, a, A, B, b, C, s, ws);
}
template <>
void gemm_hhat_t<float>(const GemmDesc& d, float a, const float* A, const float* B, float b, float* C,
                        hipStream_t s, Workspace ws) {
  gemm_f32_hhat(d, a, A, B, b, C, s, ws);
}
inline void tau_strip_t(const double* S, int o, int v, int k0, int ib, const double* eo, const double* ev, double* tau,
                        long, hipStream_t s) {
  tau_strip(S, o, v, k0, ib, eo, ev, tau, nullptr, nullptr, nullptr, nullptr, s);
}
inline void tau_strip_t(const float* S, int o, int v, int k0, int ib, const double* eo, const double* ev, float* tau,
                        long ld, hipStream_t s) {
  tau_strip_f32(S, o, v, k0, ib, eo, ev, tau, ld, s);
}

// Operands and workspace of one precision.
// ldG: row stride of G (rows (q,P)); ldtau: row stride of the stored amplitudes tau;
// ldst: row stride of the amplitude strips tau_w.  With sbf, tau, tau_w and G are the
// split-BF16 operands of the amplitude contraction (G split in place once built) and the
// strips' integrals come from BovT (B^ov transposed, split, rows of X8 values).
template <typename T>
struct Ops {
  const T *Bov, *BovLam, *Boo, *Bvv, *Boo_t, *R, *tau, *Gv, *Ev, *Go, *Eo;
  T *c, *G, *U, *H, *S, *tau_w;
  long ldG, ldtau, ldst;
  bool sbf;
  const T* BovT;
};

Ops<double> ops64(Context& c) {
  return Ops<double>{c.Bov, c.BovLam, c.Boo, c.Bvv, c.Boo_t, c.R, c.tau, c.Gv, c.Ev, c.Go, c.Eo,
                     c.w_c, c.w_G, c.w_U, c.w_H, c.w_S, c.w_tau, c.N, c.N, c.N, false, nullptr};
}
Ops<float> ops32(Context& c) {
  const bool sbf = c.split_bf16 && c.order >= 2;
  return Ops<float>{c.BovLam32, c.BovLam32, c.Boo32, c.Bvv32, c.Boo_t32, c.R32, sbf ? c.tau_sbf : c.tau32, c.Gv32,
                    c.Ev32, c.Go32, c.Eo32, c.w32_c, c.w32_G, c.w32_U, c.w32_H, c.w32_S, c.w32_tau,
                    c.N8, sbf ? c.N8 : c.N, c.N8, sbf, c.BovT_sbf};
}

// A product pass as a sequence of steps: launched as they are issued, or recorded
// (tape) so that the passes of several systems can be replayed in lockstep with the
// GEMMs of one step merged into grouped launches.
struct Step {
  int kind = 2;  // 0: FP64 GEMM, 1: FP32 GEMM, 2: any other launch
  GemmCall<double> g64;
  GemmCall<float> g32;
  std::function<void(hipStream_t)> fn;
};

template <typename T>
struct Emit {
  hipStream_t s = nullptr;
  std::vector<Step>* tape = nullptr;
  void gemm(const GemmDesc& d, T a, const T* A, const T* B, T b, T* C, Workspace ws, int tag = 0) {
    if (!tape) {
      if (tag >= 2)
        gemm_sbf16_t(d, a, A, B, b, C, s, tag == 3);
      else if (tag == 1)
        gemm_hhat_t<T>(d, a, A, B, b, C, s, ws);
      else
        gemm_t<T>(d, a, A, B, b, C, s, ws);
      return;
    }
    Step st;
    GemmCall<T> g;
    g.d = d;
    g.alpha = a;
    g.beta = b;
    g.A = A;
    g.B = B;
    g.C = C;
    g.ws = ws;
    g.tag = tag;
    put(st, g);
    tape->push_back(std::move(st));
  }
  void call(std::function<void(hipStream_t)> f) {
    if (!tape) {
      f(s);
      return;
    }
    Step st;
    st.fn = std::move(f);
    tape->push_back(std::move(st));
  }

 private:
  static void put(Step& st, const GemmCall<double>& g) {
    st.kind = 0;
    st.g64 = g;
  }
  static void put(Step& st, const GemmCall<float>& g) {
    st.kind = 1;
    st.g32 = g;
  }
};

// Every contraction of the product (see the file comment): AV <- -K_A(V) [+0],
// BV <- -K_B(V) - ring terms + ladder/ring-K terms, J, P1..P4 (delta-type
// intermediates).  The diagonal term and the final combination are done in FP64
// by sigma_assemble.
template <typename T>
void contract(Context& c, const Ops<T>& t, Emit<T>& e, int order, int k, const T* V, T* AV, T* BV, T* J, T* P1,
              T* P2, T* P3, T* P4, const PassRange& rg) {
  hipStream_t s = e.s;
  const int o = c.o, v = c.v, X = c.naux;
  const long N = c.N;
  const T one = T(1), zero = T(0), mone = T(-1);
  constexpr bool fp32 = sizeof(T) == sizeof(float);
  if (rg.pre) {
  // J: c[P][q] = sum_ia Bov[P][ia] V[q][ia];  J[q][ia] = sum_P c[P][q] Bov[P][ia]
  e.gemm(gd(X, k, (int)N, 0, N, 1, N, k), one, t.Bov, V, zero, t.c, c.ws);
  e.gemm(gd(k, (int)N, X, 1, k, 0, N, N), one, t.c, t.Bov, zero, J, c.ws);
  // G1[q][P][j][d] = sum_b V[q][j][b] Bvv[P][b][d].  B^vv_P is symmetric, so Bvv read as
  // [(P,d)][b] is the k-contiguous right operand of one GEMM with rows (q,j) = k o and
  // columns (P,d) = X v; the C index split writes row (q,j) at q X N + j v and column
  // (P,d) at P N + d, i.e. into the [q][P][j][d] layout.
  {
    GemmDesc d = gd(k * o, X * v, v, 0, v, 1, v, v);
    d.cRm = o;
    d.cSm = (long)X * t.ldG;
    d.cRn = v;
    d.cSn = t.ldG;
    e.gemm(d, one, V, t.Bvv, zero, t.G, c.ws);
  }
  // AV = -K_A(V) = -sum_P Boo_P G1_P
  {
    GemmDesc d = gd(o, v, o, 0, o, 0, v, v);
    d.KB = X;
    d.sAk = (long)o * o;
    d.sBk = t.ldG;
    d.nb1 = k;
    d.sB1 = (long)X * t.ldG;
    d.sC1 = N;
    e.gemm(d, mone, t.Boo, t.G, zero, AV, c.ws);
  }
  // U[(q,j)][(s,P,i)] = sum_b V[(q,j)][b] BovLam[(s,P,i)][b], stored as [j][(s,P)][q][i]
  // (row (q,j) of the product at q o + j Ucols k, column ((s,P),i) at (s,P) k o + i) so
  // that BV = -sum U R reads it with uniform rows (q,i)
  const int ns = order >= 2 ? 2 : 1;
  {
    const long Ucols = (long)ns * X * o;
    {
      GemmDesc d = gd(k * o, (int)Ucols, v, 0, v, 1, v, Ucols * k);
      d.cRm = o;
      d.cSm = o;
      d.cRn = o;
      d.cSn = (long)k * o;
      e.gemm(d, one, V, t.BovLam, zero, t.U, c.ws);
    }
    if (ns == c.ns) {
      // one GEMM over rows (q,i); in FP64 with the reduction splits the same product
      // batched over q would take (identical sums and rounding), in FP32 its own
      GemmDesc bq = gd(o, v, o * ns * X, 1, o, 0, v, v);
      bq.nb1 = k;
      GemmDesc d = gd(k * o, v, o * ns * X, 1, (long)k * o, 0, v, v);
      d.tile = 64;
      d.splitk = gemm_auto_splitk(fp32 ? d : bq, c.ws.bytes, fp32);
      e.gemm(d, mone, t.U, t.R, zero, BV, c.ws);
    } else {
      // first-order product on a second-order handle: K_B(V) = sum_(j,P) U[j][P][q][i] Bov[P][j][a],
      // with R[j][1][P][a] = Bov[P][j][a] (outer loop over j, inner P)
      GemmDesc d = gd(o, v, X, 1, (long)k * o, 0, v, v);
      d.KB = o;
      d.sAk = Ucols * k;
      d.sBk = (long)c.ns * X * v;
      d.nb1 = k;
      d.sA1 = o;
      d.sC1 = N;
      e.gemm(d, mone, t.U, t.R + (size_t)X * v, zero, BV, c.ws);
    }
  }
  }  // rg.pre
  if (order < 2) return;
  if (rg.pre) {
  // G_P = V Bvv_P - Boo_P V  (in place on G1)
  {
    GemmDesc d = gd(o, v, o, 0, o, 0, v, v);
    d.nb1 = k;
    d.nb2 = X;
    d.sA2 = (long)o * o;
    d.sB1 = N;
    d.sC1 = (long)X * t.ldG;
    d.sC2 = t.ldG;
    e.gemm(d, mone, t.Boo, V, one, t.G, c.ws);
  }
  if (t.sbf) {
    // G is complete: split it in place for the split-BF16 amplitude products
    T* G = t.G;
    const long n = (long)k * X * t.ldG;
    e.call([=](hipStream_t st) { split_sbf16(n, reinterpret_cast<float*>(G), st); });
  }
  // delta-type terms: P1 = V Gv, P2 = V Ev, P3 = Go V, P4 = Eo V
  e.gemm(gd(k * o, v, v, 0, v, 0, v, v), one, V, t.Gv, zero, P1, c.ws);
  e.gemm(gd(k * o, v, v, 0, v, 0, v, v), one, V, t.Ev, zero, P2, c.ws);
  {
    GemmDesc d = gd(o, v, o, 0, o, 0, v, v);
    d.nb1 = k;
    d.sB1 = N;
    d.sC1 = N;
    e.gemm(d, one, t.Go, V, zero, P3, c.ws);
    e.gemm(d, one, t.Eo, V, zero, P4, c.ws);
  }
  }  // rg.pre
  const long kX = (long)k * X;
  // H = tau G is written as [q][(i,c)][P] for the ib occupied rows i of the strip (the
  // C index split sends column (q,P) of the product to q ib v X + P), so that both outputs
  // read it with uniform strides.
  auto outputs = [&](const T* H, int i0, int ib) {
    const long hq = (long)ib * v * X;
    // BV[q][i][a] += sum_(c,P) H[q][(i,c)][P] Bvv[P][c][a]: one GEMM with rows (q,i),
    // written at q N + (i0 + i) v.  In FP64 its reduction splits are those the same
    // product batched over q would take, so every element is summed and rounded alike; in
    // FP32 it takes its own (with few rows, k ib = 128 at 256/1024/4096, the batched
    // form's split would leave the GEMM on 32 workgroups).
    {
      GemmDesc bq = gd(ib, v, X, 0, (long)v * X, 0, (long)v * v, v);
      bq.KB = v;
      bq.sAk = X;
      bq.sBk = v;
      bq.nb1 = k;
      GemmDesc d = gd(k * ib, v, X, 0, (long)v * X, 0, (long)v * v, v);
      d.KB = v;
      d.sAk = X;
      d.sBk = v;
      d.cRm = ib;
      d.cSm = N;
      d.tile = 64;
      d.splitk = gemm_auto_splitk(fp32 ? d : bq, c.ws.bytes, fp32);
      e.gemm(d, one, H, t.Bvv, one, BV + (size_t)i0 * v, c.ws);
    }
    // BV[q][i][a] -= sum_(kk,P) Boo[P][i][kk] H[q][(kk,a)][P]   kk in i0..i0+ib-1
    {
      GemmDesc d = gd(o, v, X, 0, (long)o * X, 1, X, v);
      d.KB = ib;
      d.sAk = X;
      d.sBk = (long)v * X;
      d.nb1 = k;
      d.sB1 = hq;
      d.sC1 = N;
      e.gemm(d, mone, t.Boo_t + (size_t)i0 * X, H, one, BV, c.ws);
    }
  };
  // the amplitude contraction: its own kernel symbol, or split-BF16 products in that mode
  const int hhat_tag = (sizeof(T) == sizeof(float) && c.split_bf16) ? 3 : 1;
  double hflops = 0.0;
  if (t.tau) {
    // stored amplitudes: the whole contraction in one GEMM, with the prologue
    if (!rg.pre) return;
    // H[q][(i,c)][P] = sum_(j,d) tau[(i,c)][(j,d)] G[(q,P)][(j,d)]
    GemmDesc d = gd((int)N, (int)kX, (int)N, 0, t.ldtau, 1, t.ldG, X);
    d.cRn = X;
    d.cSn = N * X;
    const int ev = (e.tape || c.no_events) ? -1 : c.events.start(s);
    e.gemm(d, one, t.tau, t.G, zero, t.H, c.ws, hhat_tag);
    if (ev >= 0) c.events.stop(ev, s, 1);
    hflops += gemm_flops(d);
    c.stats.hhat_launches += 1;
    outputs(t.H, 0, o);
  } else {
    const int ib = c.strip_rows;
    const int r1 = std::min(rg.i1 < 0 ? o : rg.i1, o);
    for (int i0 = std::max(rg.i0, 0); i0 < r1; i0 += ib) {
      const int nb = std::min(ib, r1 - i0);
      if (t.sbf) {
        // (kx|ly) of the strip rows from the split transposed B^ov (rows of X8 values)
        const long lx = c.X8;
        e.gemm(gd(nb * v, (int)N, X, 0, lx, 1, lx, N), one, t.BovT + (size_t)i0 * v * lx, t.BovT, zero, t.S, c.ws,
               2);
      } else {
        e.gemm(gd(nb * v, (int)N, X, 1, N, 0, N, N), one, t.Bov + (size_t)i0 * v, t.Bov, zero, t.S, c.ws);
      }
      {
        const T* Sst = t.S;
        T* tw = t.tau_w;
        const double *eo = c.eps_o, *evv = c.eps_v;
        const long ldst = t.ldst;
        const bool sbf = t.sbf;
        e.call([=](hipStream_t st) {
          tau_strip_t(Sst, o, v, i0, nb, eo, evv, tw, ldst, st);
          if (sbf) split_sbf16((long)nb * v * ldst, reinterpret_cast<float*>(tw), st);
        });
      }
      GemmDesc d = gd(nb * v, (int)kX, (int)N, 0, t.ldst, 1, t.ldG, X);
      d.cRn = X;
      d.cSn = (long)nb * v * X;
      const int ev = (e.tape || c.no_events) ? -1 : c.events.start(s);
      e.gemm(d, one, t.tau_w, t.G, zero, t.H, c.ws, hhat_tag);
      if (ev >= 0) c.events.stop(ev, s, 1);
      hflops += gemm_flops(d);
      c.stats.hhat_launches += 1;
      outputs(t.H, i0, nb);
    }
  }
  c.stats.hhat_flops += hflops;
}

}  // namespace

Footprint context_footprint(int o, int v, int X, int order, bool dip, bool store, int strip_rows, bool want_f32,
                            int k, bool split) {
  // mirrors setup_context, grow_workspace and grow_workspace32 (arena blocks are
  // rounded to 256 B)
  auto r = [](size_t bytes) { return ((bytes + 255) / 256) * 256; };
  const size_t D = sizeof(double), F = sizeof(float);
  const size_t N = (size_t)o * v, K = (size_t)k;
  const size_t N8 = (size_t)padded_stride((long)N), X8 = ((size_t)X + 7) / 8 * 8;
  const size_t ns = order >= 2 ? 2 : 1;
  const int ib = order >= 2 ? std::max(1, std::min(strip_rows > 0 ? strip_rows : o, o)) : 0;
  size_t keep = r(o * D) + r(v * D) + r(X * (size_t)o * o * D) + r(X * (size_t)v * v * D) + r(ns * X * N * D);
  if (dip) keep += r(3 * N * D);
  keep += r((size_t)o * o * X * D);
  keep += r(std::max<size_t>((size_t)64 << 20, (size_t)X * 1024 * D));
  keep += 3 * r(N * D);
  size_t temp = 2 * r(N * D);  // diagonal integrals, freed after setup
  if (order >= 2) {
    keep += 2 * r((size_t)v * v * D) + 2 * r((size_t)o * o * D);
    if (store) keep += r(N * N * D);
    const size_t strip = (size_t)ib * v * N * D;
    temp += (store ? 4 : 5) * r(strip);
    temp += r((size_t)tau_blocks(o, v, ib) * ((o + ib - 1) / ib) * D) + r(D);
  }
  keep += r((size_t)o * ns * X * v * D);
  if (want_f32 && order >= 1) {
    keep += r(ns * X * N * F) + 2 * r((size_t)X * o * o * F) + r((size_t)X * v * v * F) + r((size_t)o * ns * X * v * F);
    if (order >= 2) {
      if (store) keep += r(N * (split ? N8 : N) * F);
      if (split && !store) keep += r(N * X8 * F);
      keep += 2 * r((size_t)v * v * F) + 2 * r((size_t)o * o * F);
    }
  }
  // product workspaces
  size_t ws = 0;
  if (order >= 1) {
    ws += r(K * N * D) + r(4 * K * N * D);
    ws += r(X * K * D) + r(K * X * N * D) + r(K * o * ns * X * o * D);
    const size_t ibw = store ? (size_t)o : (size_t)ib;
    if (order >= 2) {
      ws += r(ibw * v * K * X * D);
      if (!store) ws += 2 * r((size_t)ib * v * N * D);
    }
    if (want_f32) {
      ws += 4 * r(K * N * F) + r(4 * K * N * F);
      ws += r(X * K * F) + r(K * X * N8 * F) + r(K * o * ns * X * o * F);
      if (order >= 2) {
        ws += r(ibw * v * K * X * F);
        if (!store) ws += r((size_t)ib * v * N * F) + r((size_t)ib * v * N8 * F);
      }
    }
  }
  return Footprint{keep + temp, keep + ws};
}

void sigma_reserve(Context& c, int k, int precision) {
  if (c.order < 1) return;
  if (precision == 1)
    grow_workspace32(c, k);
  else
    grow_workspace(c, k);
}

size_t sigma_reserve_bytes(const Context& c, int k, int precision) {
  // mirrors grow_assembly, grow_workspace and grow_workspace32: a buffer that grows is
  // freed and allocated again, so each adds its new size less its old one; the strip
  // buffers (independent of k) are allocated by the first growth only
  if (c.order < 1 || k < 1) return 0;
  auto r = [](size_t n, size_t e) { return ((n * e + 255) / 256) * 256; };
  const size_t D = sizeof(double), F = sizeof(float);
  const size_t o = c.o, v = c.v, X = c.naux, N = c.N, N8 = c.N8, ns = c.ns;
  auto grow = [&](int cap, auto per_k) -> size_t {
    if (k <= cap) return 0;
    return per_k((size_t)k) - (cap > 0 ? per_k((size_t)cap) : 0);
  };
  size_t t = grow(c.kcap_asm, [&](size_t q) { return r(q * N, D) + r(4 * q * N, D); });
  if (precision == 1) {
    const bool stored = amplitudes_stored(c, 1);
    const size_t ib = stored ? o : (size_t)c.strip_rows;
    t += grow(c.kcap32, [&](size_t q) {
      size_t b = 4 * r(q * N, F) + r(4 * q * N, F) + r(X * q, F) + r(q * X * N8, F) + r(q * o * ns * X * o, F);
      if (c.order >= 2) b += r(ib * v * q * X, F);
      return b;
    });
    if (c.kcap32 == 0 && c.order >= 2 && !stored)
      t += r((size_t)c.strip_rows * v * N, F) + r((size_t)c.strip_rows * v * N8, F);
  } else {
    const size_t ib = c.tau ? o : (size_t)c.strip_rows;
    t += grow(c.kcap, [&](size_t q) {
      size_t b = r(X * q, D) + r(q * X * N, D) + r(q * o * ns * X * o, D);
      if (c.order >= 2) b += r(ib * v * q * X, D);
      return b;
    });
    if (c.kcap == 0 && c.order >= 2 && !c.tau) t += 2 * r((size_t)c.strip_rows * v * N, D);
  }
  return t;
}

namespace {

void emit_products(Context& c, int order, int k, int prec, const double* V, double* AV, double* BV, double* SV,
                   hipStream_t s, std::vector<Step>* tape, const PassRange& rg);

// One product pass of k vectors (contractions in the given precision, then the FP64
// diagonal term and combination), launched on s or recorded on a tape; rg selects the
// part of the pass.
void emit_pass(Context& c, int order, int k, int prec, const double* V, double* AV, double* BV, double* SV,
               hipStream_t s, std::vector<Step>* tape, const PassRange& rg = PassRange{}) {
  emit_products(c, order, k, prec, V, AV, BV, SV, s, tape, rg);
  if (c.tda && rg.post) {
    // Tamm-Dancoff: B = 0
    Emit<double> em;
    em.s = s;
    em.tape = tape;
    const long n = (long)k * c.N;
    em.call([=](hipStream_t st) { fill_zero(n, BV, st); });
  }
}

void emit_products(Context& c, int order, int k, int prec, const double* V, double* AV, double* BV, double* SV,
                   hipStream_t s, std::vector<Step>* tape, const PassRange& rg) {
  const int o = c.o, v = c.v;
  const long N = c.N, kN = (long)k * N;
  const double *eo = c.eps_o, *ev = c.eps_v;
  if (order == 0) {
    if (!rg.post) return;
    Emit<double> em;
    em.s = s;
    em.tape = tape;
    em.call([=](hipStream_t st) {
      sigma_assemble(o, v, k, 0, eo, ev, V, nullptr, nullptr, nullptr, nullptr, nullptr, AV, BV, SV, st);
    });
    return;
  }
  double* J = c.w_J;
  double* Q1 = c.w_P;
  if (prec == 1) {
    if (!c.BovLam32) throw NotSupported("FP32 products need precision = PP_FP32 at setup");
    grow_workspace32(c, k);
    J = c.w_J;
    Q1 = c.w_P;
    Emit<float> em;
    em.s = s;
    em.tape = tape;
    float *V32 = c.w32_V, *AV32 = c.w32_AV, *BV32 = c.w32_BV, *J32 = c.w32_J, *P32 = c.w32_P;
    if (rg.pre) em.call([=](hipStream_t st) { to_f32(kN, V, V32, st); });
    contract<float>(c, ops32(c), em, order, k, V32, AV32, BV32, J32, P32, P32 + kN, P32 + 2 * kN, P32 + 3 * kN, rg);
    if (!rg.post) return;
    // the diagonal (orbital-energy) term and the combination stay in FP64
    em.call([=](hipStream_t st) {
      to_f64(kN, AV32, AV, st);
      to_f64(kN, BV32, BV, st);
      to_f64(kN, J32, J, st);
      if (order >= 2) to_f64(4 * kN, P32, Q1, st);
      sigma_assemble(o, v, k, order, eo, ev, V, J, Q1, Q1 + kN, Q1 + 2 * kN, Q1 + 3 * kN, AV, BV, SV, st);
    });
  } else {
    grow_workspace(c, k);
    J = c.w_J;
    Q1 = c.w_P;
    Emit<double> em;
    em.s = s;
    em.tape = tape;
    contract<double>(c, ops64(c), em, order, k, V, AV, BV, J, Q1, Q1 + kN, Q1 + 2 * kN, Q1 + 3 * kN, rg);
    if (!rg.post) return;
    em.call([=](hipStream_t st) {
      sigma_assemble(o, v, k, order, eo, ev, V, J, Q1, Q1 + kN, Q1 + 2 * kN, Q1 + 3 * kN, AV, BV, SV, st);
    });
  }
}

void pass_on_stream(Context& c, int order, int k, int prec, const double* V, double* AV, double* BV, double* SV,
                    const PassRange& rg) {
  if (order > c.order) throw InvalidArg("requested order exceeds the setup order");
  if (k <= 0) return;
  hipStream_t s = c.stream;
  if (rg.pre) ++c.pass_serial;
  if (order == 0) {
    emit_pass(c, 0, k, prec, V, AV, BV, SV, s, nullptr, rg);
    return;
  }
  if (c.no_events) {
    emit_pass(c, order, k, prec, V, AV, BV, SV, s, nullptr, rg);
  } else {
    if (c.events.pending() > 4096) c.resolve_stats();
    const int ev_pass = c.events.start(s);
    emit_pass(c, order, k, prec, V, AV, BV, SV, s, nullptr, rg);
    c.events.stop(ev_pass, s, 0);
  }
  const int r0 = std::max(rg.i0, 0), r1 = std::min(rg.i1 < 0 ? c.o : rg.i1, c.o);
  double pre, strips;
  pass_flops(c, order, k, prec, std::max(0, r1 - r0), &pre, &strips);
  const double f = (rg.pre ? pre : 0.0) + strips;
  c.stats.flops += f;
  if (prec == 1) c.stats.flops32 += f;
  if (rg.pre) c.stats.vectors += k;
}

}  // namespace

void sigma_core(Context& c, int order, int k, const double* V, double* AV, double* BV, double* SV) {
  pass_on_stream(c, order, k, 0, V, AV, BV, SV, PassRange{});
}

void sigma_core_f32(Context& c, int order, int k, const double* V, double* AV, double* BV, double* SV) {
  pass_on_stream(c, order, k, 1, V, AV, BV, SV, PassRange{});
}

bool sigma_workspace_ready(const Context& c, int order, int k, int prec) {
  if (order < 1) return true;
  if (k > c.kcap_asm) return false;
  return prec == 1 ? k <= c.kcap32 : k <= c.kcap;
}

void sigma_pass(Context& c, int order, int k, int prec, const double* V, double* AV, double* BV, double* SV,
                const PassRange& rg) {
  if (prec == 1 && !c.BovLam32 && order >= 1) throw NotSupported("reduced-precision products need a handle set up "
                                                                 "with PP_FP32 or PP_SPLIT_BF16");
  pass_on_stream(c, order, k, prec, V, AV, BV, SV, rg);
}

int sigma_group(const std::vector<PassJob>& jobs, hipStream_t s) {
  for (const PassJob& pj : jobs) ++pj.c->pass_serial;
  std::vector<std::vector<Step>> tapes(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) {
    const PassJob& pj = jobs[j];
    for (size_t i = 0; i < j; ++i)
      if (jobs[i].c == pj.c) throw InvalidArg("sigma_group: one pass per system (workspaces are per system)");
    if (pj.order > pj.c->order) throw InvalidArg("requested order exceeds the setup order");
    if (pj.k <= 0) continue;
    emit_pass(*pj.c, pj.order, pj.k, pj.prec, pj.V, pj.AV, pj.BV, pj.SV, s, &tapes[j]);
    if (pj.order >= 1) {
      pj.c->stats.flops += sigma_flops(*pj.c, pj.order, pj.k, pj.prec);
      if (pj.prec == 1) pj.c->stats.flops32 += sigma_flops(*pj.c, pj.order, pj.k, pj.prec);
      pj.c->stats.vectors += pj.k;
    }
  }
  // lockstep replay: step p of every pass, GEMMs of one step merged by tile shape
  size_t len = 0;
  for (auto& t : tapes) len = std::max(len, t.size());
  std::vector<GemmCall<double>> g64;
  std::vector<GemmCall<float>> g32;
  int grouped = 0;
  for (size_t p = 0; p < len; ++p) {
    g64.clear();
    g32.clear();
    for (auto& t : tapes) {
      if (p >= t.size()) continue;
      Step& st = t[p];
      // a GEMM whose reduction splits the launch would choose by itself is issued without
      // split-K, grouped or not, so that each system's products round the same way
      // whichever systems share the pass (fixed splits are kept)
      if (st.kind == 0) {
        g64.push_back(st.g64);
        if (g64.back().d.splitk == 0) g64.back().d.splitk = 1;
      } else if (st.kind == 1) {
        g32.push_back(st.g32);
        if (g32.back().d.splitk == 0) g32.back().d.splitk = 1;
      } else {
        st.fn(s);
      }
    }
    if (!g64.empty()) grouped += gemm_group_f64(g64, s);
    if (!g32.empty()) grouped += gemm_group_f32(g32, s);
  }
  return grouped;
}

}  // namespace ppw
