// C ABI of the ppwin library: argument checks, error translation, host<->device
// marshalling.  No exception leaves this file.
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ppwin.h"
#include "../../include/ppwin_testing.h"
#include "context.h"
#include "kernels.h"
#include "riesz.h"
#include "solver.h"
#include "abi.h"

struct pp_handle {
  ppw::Context* ctx = nullptr;
  pp_options opt{};
  std::string err;
  // staging buffers of asynchronous products (V, AV, BV, SV), kept until pp_destroy
  double* abuf = nullptr;
  size_t acap = 0;     // doubles per buffer
  bool pending = false;  // asynchronous work may still be running on the handle's stream
  // a product pass issued in parts (pp_sigma_part): its arguments, staging (V, AV, BV, SV
  // and, for host output, out) and the next part expected
  struct Parts {
    int next = -1;  // -1: no pass in progress
    int order = 0, m = 0, n_parts = 0;
    const double* X = nullptr;
    double* out = nullptr;
    uint32_t flags = 0;
    long serial = 0;
    double* buf = nullptr;
    double* dout = nullptr;
  } parts;
};

namespace {
std::atomic<long> g_inject_countdown{0};
std::atomic<int> g_inject_code{0};
}  // namespace

namespace ppw {
hipError_t injected_hip_error(hipError_t e) {
  if (g_inject_countdown.load(std::memory_order_relaxed) > 0 && g_inject_countdown.fetch_sub(1) == 1)
    return static_cast<hipError_t>(g_inject_code.load());
  return e;
}
}  // namespace ppw

namespace {

thread_local std::string g_setup_error;
using ppw::guarded;

// Staging of pp_sigma_static: a fixed device array, one copy per GPU, shared by every
// call on that GPU (calls that overlap on one GPU race).  Host code never passes the
// array's name to a kernel: it uses the device address taken once per device with
// hipGetSymbolAddress.
constexpr size_t kScratchDoubles = (size_t)8 << 20;  // 64 MiB
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (the device must be current).
double* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) throw ppw::InvalidArg("device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    PPW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw ppw::DeviceError("hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  return g_scratch_ptr[device];
}

}  // namespace

namespace {
// Waits for asynchronous products still running on the handle's stream, so that the
// caller's next call (whatever streams it uses) finds their buffers settled.
void settle(pp_handle* h) {
  if (h->pending) {
    PPW_HIP(hipSetDevice(h->ctx->device));
    PPW_HIP(hipStreamSynchronize(h->ctx->stream));
    h->pending = false;
  }
}

// Drops the staging of a pass issued in parts (after its work is settled).
void drop_parts(pp_handle* h) {
  if (h->parts.buf) h->ctx->arena.free(h->parts.buf);
  if (h->parts.dout) h->ctx->arena.free(h->parts.dout);
  h->parts = pp_handle::Parts{};
}

// Precision of the contractions a product call asks for (PP_REDUCED: the handle's).
int product_precision(const pp_handle* h, uint32_t flags) {
  if (!(flags & PP_REDUCED)) return 0;
  if (h->opt.precision == PP_FP64)
    throw ppw::NotSupported("PP_REDUCED needs a handle set up with PP_FP32 or PP_SPLIT_BF16");
  return 1;
}
}  // namespace

extern "C" {

void pp_default_options(pp_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = PP_FP64;
  opt->store_amplitudes = -1;
  opt->strip_rows = 0;
  opt->tol = 1e-9;
  opt->block = 0;
  opt->krylov_steps = 2;
  opt->max_basis = 480;
  opt->max_cycles = 200;
  opt->d_clamp = 1e-4;
  opt->hbm_budget = 0;
  opt->device = 0;
  opt->stream = nullptr;
  opt->seed = 0;
  opt->method = PP_FOLDED;
  opt->contour_nodes = 6;
  opt->contour_tol = 1e-4;
  opt->contour_maxit = 500;
  opt->pass_vectors = 0;
}

pp_status pp_setup(const pp_system* sys, const pp_options* opt_in, pp_handle** out) {
  if (out) *out = nullptr;
  g_setup_error.clear();
  pp_handle* h = nullptr;
  pp_status st = guarded(&g_setup_error, [&] {
    if (!sys || !out) throw ppw::InvalidArg("sys and out must not be NULL");
    pp_options opt;
    pp_default_options(&opt);
    if (opt_in) opt = *opt_in;
    ppw::check_options(opt);
    const int o = sys->n_occ, v = sys->n_vir, X = sys->n_aux;
    if (o < 1 || v < 1 || X < 1) throw ppw::InvalidArg("n_occ, n_vir and n_aux must be positive");
    if (!sys->eps || !sys->B_oo || !sys->B_ov || !sys->B_vv) throw ppw::InvalidArg("NULL input array");
    if (!sys->device_ptrs) ppw::check_host_system(*sys);
    ppw::SetupParams p;
    p.o = o;
    p.v = v;
    p.naux = X;
    p.order = sys->order;
    p.eps = sys->eps;
    p.Boo = sys->B_oo;
    p.Bov = sys->B_ov;
    p.Bvv = sys->B_vv;
    p.dip = sys->dip;
    p.device_ptrs = sys->device_ptrs != 0;
    p.store_amplitudes = opt.store_amplitudes;
    p.strip_rows = opt.strip_rows;
    p.want_f32 = opt.precision != PP_FP64;
    p.split_bf16 = opt.precision == PP_SPLIT_BF16;
    p.tda = opt.tda != 0;
    p.budget = opt.hbm_budget;
    p.device = opt.device;
    p.stream = static_cast<hipStream_t>(opt.stream);
    h = new pp_handle();
    h->opt = opt;
    h->ctx = ppw::setup_context(p);
    *out = h;
  });
  if (st != PP_OK && h) {
    delete h->ctx;
    delete h;
    if (out) *out = nullptr;
  }
  return st;
}

pp_status pp_sigma(pp_handle* h, int32_t order, int32_t m, const double* X, double* outp, uint32_t flags) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    ppw::Context& c = *h->ctx;
    if (m < 0) throw ppw::InvalidArg("m must be >= 0");
    if (order < 0 || order > c.order) throw ppw::InvalidArg("order exceeds the setup order");
    if (m == 0) return;
    if (!X || !outp) throw ppw::InvalidArg("NULL vector pointer");
    PPW_HIP(hipSetDevice(c.device));
    const long N = c.N;
    const bool dev = (flags & PP_DEVICE_PTRS) != 0;
    const bool async = (flags & PP_ASYNC) != 0;
    if (async && !dev) throw ppw::InvalidArg("PP_ASYNC needs PP_DEVICE_PTRS");
    (void)product_precision(h, flags);
    const int k = 2 * m;
    const size_t per = (size_t)k * N;
    struct Free {
      ppw::Context& c;
      std::vector<void*> p;
      ~Free() {
        for (void* q : p) c.arena.free(q);
      }
    } fr{c, {}};
    double *V, *AV, *BV, *SV;
    if (async) {
      // handle-owned staging, grown only after earlier asynchronous work is done
      if (per > h->acap) {
        settle(h);
        if (h->abuf) c.arena.free(h->abuf);
        h->abuf = nullptr;
        h->acap = 0;
        h->abuf = c.arena.alloc<double>(4 * per, "async sigma staging");
        h->acap = per;
      }
      V = h->abuf;
      AV = V + h->acap;
      BV = AV + h->acap;
      SV = BV + h->acap;
    } else {
      settle(h);
      V = c.arena.alloc<double>(per, "sigma V");
      fr.p.push_back(V);
      AV = c.arena.alloc<double>(per, "sigma AV");
      fr.p.push_back(AV);
      BV = c.arena.alloc<double>(per, "sigma BV");
      fr.p.push_back(BV);
      SV = c.arena.alloc<double>(per, "sigma SV");
      fr.p.push_back(SV);
    }
    double* out = outp;
    if (!dev) {
      out = c.arena.alloc<double>((size_t)2 * m * N, "sigma out");
      fr.p.push_back(out);
    }
    const hipMemcpyKind kin = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    PPW_HIP(hipMemcpy2DAsync(V, N * sizeof(double), X, 2 * N * sizeof(double), N * sizeof(double), m, kin,
                             c.stream));
    PPW_HIP(hipMemcpy2DAsync(V + (size_t)m * N, N * sizeof(double), X + N, 2 * N * sizeof(double),
                             N * sizeof(double), m, kin, c.stream));
    const bool metric = (flags & PP_APPLY_METRIC) != 0;
    ppw::sigma_pass(c, order, k, product_precision(h, flags), V, AV, BV, SV, ppw::PassRange{});
    ppw::combine_pairs(N, m, AV, BV, SV, metric, out, c.stream);
    if (!dev)
      PPW_HIP(hipMemcpyAsync(outp, out, sizeof(double) * 2 * m * N, hipMemcpyDeviceToHost, c.stream));
    if (async) {
      h->pending = true;
      return;
    }
    PPW_HIP(hipStreamSynchronize(c.stream));
  });
}

pp_status pp_sigma_part(pp_handle* h, int32_t order, int32_t m, const double* X, double* outp, uint32_t flags,
                        int32_t part, int32_t n_parts) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    ppw::Context& c = *h->ctx;
    pp_handle::Parts& ps = h->parts;
    if (n_parts < 1 || n_parts > c.o) throw ppw::InvalidArg("n_parts must be in 1..n_occ");
    if (part < 0 || part >= n_parts) throw ppw::InvalidArg("part must be in 0..n_parts-1");
    if (m < 1) throw ppw::InvalidArg("m must be >= 1");
    if (order < 0 || order > c.order) throw ppw::InvalidArg("order exceeds the setup order");
    if (!X || !outp) throw ppw::InvalidArg("NULL vector pointer");
    const bool dev = (flags & PP_DEVICE_PTRS) != 0;
    const bool async = (flags & PP_ASYNC) != 0;
    if (async && !dev) throw ppw::InvalidArg("PP_ASYNC needs PP_DEVICE_PTRS");
    const int prec = product_precision(h, flags);
    PPW_HIP(hipSetDevice(c.device));
    const long N = c.N;
    const int k = 2 * m;
    const size_t per = (size_t)k * N;
    if (part == 0) {
      settle(h);
      drop_parts(h);
      ps.buf = c.arena.alloc<double>(4 * per, "sigma part staging");
      if (!dev) ps.dout = c.arena.alloc<double>((size_t)2 * m * N, "sigma part out");
      ps.order = order;
      ps.m = m;
      ps.n_parts = n_parts;
      ps.X = X;
      ps.out = outp;
      ps.flags = flags;
    } else {
      if (ps.next < 0) throw ppw::InvalidArg("no product pass in parts is in progress: start at part 0");
      if (part != ps.next || order != ps.order || m != ps.m || n_parts != ps.n_parts || X != ps.X ||
          outp != ps.out || flags != ps.flags)
        throw ppw::InvalidArg("parts of a pass must come in order with the arguments of its part 0");
      if (c.pass_serial != ps.serial) {
        settle(h);
        drop_parts(h);
        throw ppw::InvalidArg("another product ran on the handle since part 0: start the pass again");
      }
    }
    double* V = ps.buf;
    double* AV = V + per;
    double* BV = AV + per;
    double* SV = BV + per;
    if (part == 0) {
      const hipMemcpyKind kin = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
      PPW_HIP(hipMemcpy2DAsync(V, N * sizeof(double), X, 2 * N * sizeof(double), N * sizeof(double), m, kin,
                               c.stream));
      PPW_HIP(hipMemcpy2DAsync(V + (size_t)m * N, N * sizeof(double), X + N, 2 * N * sizeof(double),
                               N * sizeof(double), m, kin, c.stream));
    }
    ppw::PassRange rg;
    rg.pre = part == 0;
    rg.post = part == n_parts - 1;
    rg.i0 = (int)((long)c.o * part / n_parts);
    rg.i1 = (int)((long)c.o * (part + 1) / n_parts);
    ppw::sigma_pass(c, order, k, prec, V, AV, BV, SV, rg);
    if (rg.post) {
      double* out = dev ? outp : ps.dout;
      ppw::combine_pairs(N, m, AV, BV, SV, (flags & PP_APPLY_METRIC) != 0, out, c.stream);
      if (!dev) PPW_HIP(hipMemcpyAsync(outp, out, sizeof(double) * 2 * m * N, hipMemcpyDeviceToHost, c.stream));
    }
    ps.serial = c.pass_serial;
    ps.next = rg.post ? -1 : part + 1;
    if (async) {
      h->pending = true;
    } else {
      PPW_HIP(hipStreamSynchronize(c.stream));
    }
    if (rg.post) {
      // the staging may still be read by enqueued work: keep it until that is settled
      if (!async) drop_parts(h);
    }
  });
}

pp_status pp_sigma_static(pp_handle* h, int32_t order, int32_t m, const double* X, double* out, uint32_t flags) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    ppw::Context& c = *h->ctx;
    if (m < 0) throw ppw::InvalidArg("m must be >= 0");
    if (order < 0 || order > c.order) throw ppw::InvalidArg("order exceeds the setup order");
    if (m == 0) return;
    if (!X || !out) throw ppw::InvalidArg("NULL vector pointer");
    if (!(flags & PP_DEVICE_PTRS)) throw ppw::InvalidArg("pp_sigma_static takes device pointers (PP_DEVICE_PTRS)");
    const int prec = product_precision(h, flags);
    const long N = c.N;
    const int k = 2 * m;
    const size_t per = (size_t)k * N;
    if (4 * per > kScratchDoubles)
      throw ppw::InvalidArg("pp_sigma_static: 4 * 2m * N = " + std::to_string(4 * per) +
                            " doubles of staging exceed its fixed scratch of " + std::to_string(kScratchDoubles));
    if (!ppw::sigma_workspace_ready(c, order, k, prec))
      throw ppw::InvalidArg("pp_sigma_static: the handle's product workspace does not hold 2m vectors at this "
                            "precision yet (one pp_sigma call with at least m vectors reserves it)");
    PPW_HIP(hipSetDevice(c.device));
    settle(h);
    double* V = scratch_on(c.device);
    double* AV = V + per;
    double* BV = AV + per;
    double* SV = BV + per;
    PPW_HIP(hipMemcpy2DAsync(V, N * sizeof(double), X, 2 * N * sizeof(double), N * sizeof(double), m,
                             hipMemcpyDeviceToDevice, c.stream));
    PPW_HIP(hipMemcpy2DAsync(V + (size_t)m * N, N * sizeof(double), X + N, 2 * N * sizeof(double),
                             N * sizeof(double), m, hipMemcpyDeviceToDevice, c.stream));
    struct Quiet {
      ppw::Context& c;
      ~Quiet() { c.no_events = false; }
    } quiet{c};
    c.no_events = true;
    ppw::sigma_pass(c, order, k, prec, V, AV, BV, SV, ppw::PassRange{});
    ppw::combine_pairs(N, m, AV, BV, SV, (flags & PP_APPLY_METRIC) != 0, out, c.stream);
    if (flags & PP_ASYNC) {
      h->pending = true;
      return;
    }
    PPW_HIP(hipStreamSynchronize(c.stream));
  });
}

pp_status pp_sync(pp_handle* h) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    PPW_HIP(hipSetDevice(h->ctx->device));
    h->pending = true;  // also waits for anything else on the stream
    settle(h);
  });
}

pp_status pp_window_solve(pp_handle* h, double omega0, int32_t n_roots, double* energies, double* vectors,
                          double* osc, pp_solve_info* info) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    if (!std::isfinite(omega0)) throw ppw::InvalidArg("omega0 must be finite");
    if (n_roots < 1 || n_roots > PP_MAX_ROOTS || n_roots > h->ctx->N)
      throw ppw::InvalidArg("n_roots out of range");
    if (!energies) throw ppw::InvalidArg("energies must not be NULL");
    if (osc && !h->ctx->dip) throw ppw::InvalidArg("oscillator strengths need dipole integrals at setup");
    const ppw::SolveOptions so = ppw::solve_options(h->opt);
    settle(h);
    ppw::window_solve(*h->ctx, so, omega0, n_roots, energies, vectors, osc, info);
  });
}

pp_status pp_window_solve_batch(pp_handle* h, int32_t n_windows, const double* omega0, int32_t n_roots,
                                double* energies, double* vectors, double* osc, pp_solve_info* info) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    if (n_windows < 1 || n_windows > 64) throw ppw::InvalidArg("n_windows must be in 1..64");
    if (!omega0 || !energies) throw ppw::InvalidArg("omega0 and energies must not be NULL");
    for (int w = 0; w < n_windows; ++w)
      if (!std::isfinite(omega0[w])) throw ppw::InvalidArg("omega0 must be finite");
    if (n_roots < 1 || n_roots > PP_MAX_ROOTS || n_roots > h->ctx->N) throw ppw::InvalidArg("n_roots out of range");
    if (osc && !h->ctx->dip) throw ppw::InvalidArg("oscillator strengths need dipole integrals at setup");
    const ppw::SolveOptions so = ppw::solve_options(h->opt);
    settle(h);
    ppw::window_solve_many(*h->ctx, so, n_windows, omega0, n_roots, energies, vectors, osc, info);
  });
}

pp_status pp_get_stats(pp_handle* h, pp_stats* st) {
  if (!h || !h->ctx || !st) return PP_EINVAL;
  return guarded(&h->err, [&] {
    PPW_HIP(hipSetDevice(h->ctx->device));
    settle(h);
    h->ctx->resolve_stats();
    const ppw::SigmaStats& s = h->ctx->stats;
    st->product_flops = s.flops;
    st->product_seconds = s.seconds;
    st->product_vectors = s.vectors;
    st->hhat_flops = s.hhat_flops;
    st->hhat_seconds = s.hhat_seconds;
    st->hhat_launches = s.hhat_launches;
  });
}

pp_status pp_reset_stats(pp_handle* h) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    settle(h);
    h->ctx->resolve_stats();
    h->ctx->stats = ppw::SigmaStats{};
  });
}

double pp_mp2_energy(const pp_handle* h) { return (h && h->ctx) ? h->ctx->emp2 : 0.0; }

uint64_t pp_device_bytes(const pp_handle* h) { return (h && h->ctx) ? h->ctx->arena.used() : 0; }

pp_status pp_destroy(pp_handle* h) {
  if (!h) return PP_OK;
  std::string dummy;
  pp_status st = guarded(&dummy, [&] {
    if (h->ctx) {
      (void)hipSetDevice(h->ctx->device);
      settle(h);
      if (h->abuf) h->ctx->arena.free(h->abuf);
      h->abuf = nullptr;
      drop_parts(h);
    }
    delete h->ctx;
    h->ctx = nullptr;
  });
  delete h;
  return st;
}

pp_status pp_exciton_dos(pp_handle* h, int32_t n_bins, const double* edges, double* counts, double* mu2) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    settle(h);
    if (n_bins < 1 || n_bins > (1 << 20)) throw ppw::InvalidArg("n_bins out of range");
    if (!edges || !counts) throw ppw::InvalidArg("edges and counts must not be NULL");
    for (int b = 0; b < n_bins; ++b)
      if (!(edges[b] < edges[b + 1])) throw ppw::InvalidArg("edges must be strictly ascending");
    ppw::Context& c = *h->ctx;
    PPW_HIP(hipSetDevice(c.device));
    double *d_edges = nullptr, *d_out = nullptr;
    PPW_HIP(hipMalloc(&d_edges, sizeof(double) * (n_bins + 1)));
    hipError_t e = hipMalloc(&d_out, sizeof(double) * 2 * n_bins);
    if (e != hipSuccess) {
      (void)hipFree(d_edges);
      PPW_HIP(e);
    }
    std::vector<double> out(2 * (size_t)n_bins);
    try {
      PPW_HIP(hipMemcpyAsync(d_edges, edges, sizeof(double) * (n_bins + 1), hipMemcpyHostToDevice, c.stream));
      ppw::exciton_dos(c.o, c.v, c.eps_o, c.eps_v, c.dip, d_edges, n_bins, d_out, c.stream);
      PPW_HIP(hipMemcpyAsync(out.data(), d_out, sizeof(double) * 2 * n_bins, hipMemcpyDeviceToHost, c.stream));
      PPW_HIP(hipStreamSynchronize(c.stream));
    } catch (...) {
      (void)hipFree(d_edges);
      (void)hipFree(d_out);
      throw;
    }
    (void)hipFree(d_edges);
    (void)hipFree(d_out);
    for (int b = 0; b < n_bins; ++b) {
      counts[b] = out[2 * b];
      if (mu2) mu2[b] = out[2 * b + 1];
    }
  });
}

namespace {
// Roots and a frequency grid (host arrays) to the current device, response_on_grid there,
// results back: Pi's real and imaginary parts and the broadened strengths (each nullable).
void grid_sums(int32_t n, const double* energies, const double* osc, int32_t n_omega, const double* omega,
               double eta, double* re, double* im, double* lor) {
  if (n_omega == 0) return;
  std::vector<double> host;  // e, f, omega
  host.insert(host.end(), energies, energies + n);
  host.insert(host.end(), osc, osc + n);
  host.insert(host.end(), omega, omega + n_omega);
  const size_t nin = host.size(), nout = (size_t)3 * n_omega;
  double* d = nullptr;
  PPW_HIP(hipMalloc(&d, sizeof(double) * (nin + nout)));
  struct Free {
    double* p;
    ~Free() { (void)hipFree(p); }
  } fr{d};
  PPW_HIP(hipMemcpy(d, host.data(), sizeof(double) * nin, hipMemcpyHostToDevice));
  double* out = d + nin;
  ppw::response_on_grid(n, d, d + n, n_omega, d + 2 * n, eta, re ? out : nullptr, im ? out + n_omega : nullptr,
                        lor ? out + 2 * n_omega : nullptr, nullptr);
  PPW_HIP(hipDeviceSynchronize());
  if (re) PPW_HIP(hipMemcpy(re, out, sizeof(double) * n_omega, hipMemcpyDeviceToHost));
  if (im) PPW_HIP(hipMemcpy(im, out + n_omega, sizeof(double) * n_omega, hipMemcpyDeviceToHost));
  if (lor) PPW_HIP(hipMemcpy(lor, out + 2 * n_omega, sizeof(double) * n_omega, hipMemcpyDeviceToHost));
}

void check_roots(int32_t n, const double* energies, const double* osc, int32_t n_omega, const double* omega) {
  if (n < 0 || n_omega < 0) throw ppw::InvalidArg("negative size");
  if ((n > 0 && (!energies || !osc)) || (n_omega > 0 && !omega)) throw ppw::InvalidArg("NULL array");
  for (int k = 0; k < n; ++k)
    if (!(energies[k] > 0.0) || !std::isfinite(energies[k]) || !std::isfinite(osc[k]))
      throw ppw::InvalidArg("energies must be positive and finite, strengths finite");
  for (int g = 0; g < n_omega; ++g)
    if (!std::isfinite(omega[g])) throw ppw::InvalidArg("non-finite frequency");
}
}  // namespace

pp_status pp_spectrum(int32_t n, const double* energies, const double* osc, int32_t n_omega, const double* omega,
                      double eta, double* out) {
  g_setup_error.clear();
  return guarded(&g_setup_error, [&] {
    check_roots(n, energies, osc, n_omega, omega);
    if (!(eta > 0.0) || !std::isfinite(eta)) throw ppw::InvalidArg("eta must be positive");
    if (n_omega > 0 && !out) throw ppw::InvalidArg("NULL array");
    grid_sums(n, energies, osc, n_omega, omega, eta, nullptr, nullptr, out);
  });
}

pp_status pp_response(int32_t n, const double* energies, const double* osc, int32_t n_omega, const double* omega,
                      double eta, double* re, double* im) {
  g_setup_error.clear();
  return guarded(&g_setup_error, [&] {
    check_roots(n, energies, osc, n_omega, omega);
    if (!(eta >= 0.0) || !std::isfinite(eta)) throw ppw::InvalidArg("eta must be >= 0 and finite");
    if (n_omega > 0 && (!re || !im)) throw ppw::InvalidArg("NULL array");
    grid_sums(n, energies, osc, n_omega, omega, eta, re, im, nullptr);
  });
}

const char* pp_status_string(pp_status s) {
  switch (s) {
    case PP_OK: return "PP_OK";
    case PP_EINVAL: return "PP_EINVAL: invalid argument";
    case PP_ENOMEM: return "PP_ENOMEM: device memory budget exceeded";
    case PP_ENOTCONV: return "PP_ENOTCONV: solve did not converge";
    case PP_EUNSTABLE: return "PP_EUNSTABLE: response matrix not positive definite";
    case PP_EDEVICE: return "PP_EDEVICE: HIP runtime error";
    case PP_ENOTSUP: return "PP_ENOTSUP: not supported";
    case PP_EPENDING: return "PP_EPENDING: request not finished";
  }
  return "unknown status";
}

const char* pp_last_error(const pp_handle* h) {
  if (!h) return g_setup_error.c_str();
  return h->err.c_str();
}

// ---------------------------------------------------------------------------
// test hooks
// ---------------------------------------------------------------------------
namespace {
// The split-BF16 GEMM on FP32 operands in the plain layout (A [M][lda], B [N][ldb], both
// contiguous along k): the operands are copied into zero-padded rows of a multiple of 8
// values, split there and multiplied.
void sbf16_from_f32(ppw::GemmDesc d, float alpha, const float* A, const float* B, float beta, float* C) {
  if (d.transA != 0 || d.transB == 0 || d.KB != 1 || d.nb1 != 1 || d.nb2 != 1)
    throw ppw::InvalidArg("split-BF16 GEMM: operands contiguous along k, no batch or outer reduction");
  if (d.M <= 0 || d.N <= 0) return;
  if (d.K <= 0) throw ppw::InvalidArg("gemm: empty reduction");
  const long ld = ((long)(d.K + 7) / 8) * 8;
  float* As = nullptr;
  float* Bs = nullptr;
  try {
    PPW_HIP(hipMalloc(&As, sizeof(float) * d.M * ld));
    PPW_HIP(hipMalloc(&Bs, sizeof(float) * d.N * ld));
    PPW_HIP(hipMemset(As, 0, sizeof(float) * d.M * ld));
    PPW_HIP(hipMemset(Bs, 0, sizeof(float) * d.N * ld));
    PPW_HIP(hipMemcpy2D(As, sizeof(float) * ld, A, sizeof(float) * d.lda, sizeof(float) * d.K, d.M,
                        hipMemcpyDeviceToDevice));
    PPW_HIP(hipMemcpy2D(Bs, sizeof(float) * ld, B, sizeof(float) * d.ldb, sizeof(float) * d.K, d.N,
                        hipMemcpyDeviceToDevice));
    ppw::split_sbf16((long)d.M * ld, As, nullptr);
    ppw::split_sbf16((long)d.N * ld, Bs, nullptr);
    d.lda = ld;
    d.ldb = ld;
    ppw::gemm_sbf16(d, alpha, As, Bs, beta, C, nullptr);
    PPW_HIP(hipDeviceSynchronize());
  } catch (...) {
    (void)hipFree(As);
    (void)hipFree(Bs);
    throw;
  }
  (void)hipFree(As);
  (void)hipFree(Bs);
}
}  // namespace

pp_status ppint_inject_hip_error(int32_t after_calls, int32_t code) {
  g_setup_error.clear();
  if (after_calls < 0 || (after_calls > 0 && code == 0)) {
    g_setup_error = "after_calls must be >= 0 and code nonzero";
    return PP_EINVAL;
  }
  g_inject_countdown.store(0);
  g_inject_code.store(code);
  g_inject_countdown.store(after_calls);
  return PP_OK;
}

pp_status ppint_split_sbf16(int64_t n, float* x) {
  g_setup_error.clear();
  return guarded(&g_setup_error, [&] {
    ppw::split_sbf16(n, x, nullptr);
    PPW_HIP(hipDeviceSynchronize());
  });
}

pp_status ppint_gemm(int32_t fp32, int32_t M, int32_t N, int32_t K, int32_t KB, int32_t nbatch, int32_t transA,
                     int64_t lda, int64_t sA, int64_t sAk, int32_t transB, int64_t ldb, int64_t sB, int64_t sBk,
                     int64_t ldc, int64_t sC, double alpha, const void* A, const void* B, double beta, void* C,
                     uint64_t ws_bytes) {
  g_setup_error.clear();
  void* ws = nullptr;
  pp_status st = guarded(&g_setup_error, [&] {
    ppw::GemmDesc d;
    d.M = M;
    d.N = N;
    d.K = K;
    d.KB = KB;
    d.nb1 = nbatch;
    d.transA = transA;
    d.lda = lda;
    d.sA1 = sA;
    d.sAk = sAk;
    d.transB = transB;
    d.ldb = ldb;
    d.sB1 = sB;
    d.sBk = sBk;
    d.ldc = ldc;
    d.sC1 = sC;
    ppw::Workspace w;
    if (ws_bytes) {
      PPW_HIP(hipMalloc(&ws, ws_bytes));
      w.ptr = ws;
      w.bytes = ws_bytes;
    }
    if (fp32 >= 3 && fp32 <= 5) {
      d.tile = fp32 == 4 ? 128 : (fp32 == 5 ? 256 : 0);
      ppw::gemm_sbf16(d, (float)alpha, (const float*)A, (const float*)B, (float)beta, (float*)C, nullptr);
    }
    else if (fp32 == 2)
      sbf16_from_f32(d, (float)alpha, (const float*)A, (const float*)B, (float)beta, (float*)C);
    else if (fp32)
      ppw::gemm_f32(d, (float)alpha, (const float*)A, (const float*)B, (float)beta, (float*)C, nullptr, w);
    else
      ppw::gemm_f64(d, alpha, (const double*)A, (const double*)B, beta, (double*)C, nullptr, w);
    PPW_HIP(hipDeviceSynchronize());
  });
  if (ws) (void)hipFree(ws);
  return st;
}

pp_status ppint_gemm_cmap(int32_t fp32, int32_t M, int32_t N, int32_t K, int32_t transA, int64_t lda, int32_t transB,
                          int64_t ldb, int64_t ldc, int32_t cRm, int64_t cSm, int32_t cRn, int64_t cSn, double alpha,
                          const void* A, const void* B, double beta, void* C, uint64_t ws_bytes) {
  g_setup_error.clear();
  void* ws = nullptr;
  pp_status st = guarded(&g_setup_error, [&] {
    ppw::GemmDesc d;
    d.M = M;
    d.N = N;
    d.K = K;
    d.transA = transA;
    d.lda = lda;
    d.transB = transB;
    d.ldb = ldb;
    d.ldc = ldc;
    d.cRm = cRm;
    d.cSm = cSm;
    d.cRn = cRn;
    d.cSn = cSn;
    ppw::Workspace w;
    if (ws_bytes) {
      PPW_HIP(hipMalloc(&ws, ws_bytes));
      w.ptr = ws;
      w.bytes = ws_bytes;
    }
    if (fp32 >= 3 && fp32 <= 5) {
      d.tile = fp32 == 4 ? 128 : (fp32 == 5 ? 256 : 0);
      ppw::gemm_sbf16(d, (float)alpha, (const float*)A, (const float*)B, (float)beta, (float*)C, nullptr);
    }
    else if (fp32 == 2)
      sbf16_from_f32(d, (float)alpha, (const float*)A, (const float*)B, (float)beta, (float*)C);
    else if (fp32)
      ppw::gemm_f32(d, (float)alpha, (const float*)A, (const float*)B, (float)beta, (float*)C, nullptr, w);
    else
      ppw::gemm_f64(d, alpha, (const double*)A, (const double*)B, beta, (double*)C, nullptr, w);
    PPW_HIP(hipDeviceSynchronize());
  });
  if (ws) (void)hipFree(ws);
  return st;
}

pp_status ppint_gemm_group(int32_t fp32, int32_t n, const ppint_gemm_member* m, int32_t* grouped_launches) {
  g_setup_error.clear();
  return guarded(&g_setup_error, [&] {
    if (n < 1 || !m) throw ppw::InvalidArg("ppint_gemm_group: no members");
    auto desc = [](const ppint_gemm_member& x) {
      ppw::GemmDesc d;
      d.M = x.M;
      d.N = x.N;
      d.K = x.K;
      d.transA = x.transA;
      d.transB = x.transB;
      d.lda = x.lda;
      d.ldb = x.ldb;
      d.ldc = x.ldc;
      return d;
    };
    int g = 0;
    if (fp32) {
      std::vector<ppw::GemmCall<float>> calls(n);
      for (int i = 0; i < n; ++i) {
        calls[i].d = desc(m[i]);
        calls[i].alpha = (float)m[i].alpha;
        calls[i].beta = (float)m[i].beta;
        calls[i].A = (const float*)m[i].A;
        calls[i].B = (const float*)m[i].B;
        calls[i].C = (float*)m[i].C;
      }
      g = ppw::gemm_group_f32(calls, nullptr);
    } else {
      std::vector<ppw::GemmCall<double>> calls(n);
      for (int i = 0; i < n; ++i) {
        calls[i].d = desc(m[i]);
        calls[i].alpha = m[i].alpha;
        calls[i].beta = m[i].beta;
        calls[i].A = (const double*)m[i].A;
        calls[i].B = (const double*)m[i].B;
        calls[i].C = (double*)m[i].C;
      }
      g = ppw::gemm_group_f64(calls, nullptr);
    }
    PPW_HIP(hipDeviceSynchronize());
    if (grouped_launches) *grouped_launches = g;
  });
}

pp_status ppint_partial_syev(int32_t n, const double* A, double target, int32_t p, double* lam, double* Z,
                             int32_t* q) {
  g_setup_error.clear();
  double* scr = nullptr;
  pp_status st = guarded(&g_setup_error, [&] {
    PPW_HIP(hipMalloc(&scr, sizeof(double) * ppw::partial_syev_scratch(n, p)));
    const int got = ppw::partial_syev(n, A, target, p, lam, Z, scr, nullptr);
    PPW_HIP(hipDeviceSynchronize());
    if (q) *q = got;
  });
  if (scr) (void)hipFree(scr);
  return st;
}

pp_status ppint_syev(int32_t n, const double* A, double* w, double* Z) {
  g_setup_error.clear();
  return guarded(&g_setup_error, [&] {
    ppw::small_syev(n, A, w, Z, nullptr);
    PPW_HIP(hipDeviceSynchronize());
  });
}

pp_status ppint_cholesky(int32_t n, const double* A, double* L) {
  g_setup_error.clear();
  return guarded(&g_setup_error, [&] {
    ppw::small_cholesky(n, A, L, nullptr, nullptr);
    PPW_HIP(hipDeviceSynchronize());
  });
}

pp_status ppint_riesz_filter(pp_handle* h, double center, double radius, int32_t nodes, double tol, int32_t maxit,
                             int32_t m, const double* V, double* out, int32_t* iters, double* worst) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    settle(h);
    ppw::Context& c = *h->ctx;
    if (m < 1 || m > 64) throw ppw::InvalidArg("m must be in 1..64");
    if (nodes < 1 || nodes > 32) throw ppw::InvalidArg("nodes must be in 1..32");
    if (!(radius > 0) || !std::isfinite(center) || !(tol > 0 && tol < 1) || maxit < 1)
      throw ppw::InvalidArg("bad contour parameters");
    if (!V || !out) throw ppw::InvalidArg("NULL vector pointer");
    PPW_HIP(hipSetDevice(c.device));
    const long N = c.N;
    double* W = c.arena.alloc<double>((size_t)2 * m * N, "riesz block");
    struct Free {
      ppw::Context& c;
      double* p;
      ~Free() { c.arena.free(p); }
    } fr{c, W};
    // [m][2][N] -> X rows then Y rows
    PPW_HIP(hipMemcpy2DAsync(W, N * sizeof(double), V, 2 * N * sizeof(double), N * sizeof(double), m,
                             hipMemcpyDeviceToDevice, c.stream));
    PPW_HIP(hipMemcpy2DAsync(W + (size_t)m * N, N * sizeof(double), V + N, 2 * N * sizeof(double),
                             N * sizeof(double), m, hipMemcpyDeviceToDevice, c.stream));
    ppw::ContourFilter cf(c, m, nodes, 2 * m, c.stream);
    ppw::ContourParams p;
    p.center = center;
    p.radius = radius;
    p.nodes = nodes;
    p.tol = tol;
    p.maxit = maxit;
    double wr = 0.0;
    const int it = cf.apply(p, m, W, [&](int k, const double* X, double* AV, double* BV, double* SV) {
      ppw::sigma_core(c, c.order, k, X, AV, BV, SV);
    }, &wr);
    PPW_HIP(hipMemcpy2DAsync(out, 2 * N * sizeof(double), W, N * sizeof(double), N * sizeof(double), m,
                             hipMemcpyDeviceToDevice, c.stream));
    PPW_HIP(hipMemcpy2DAsync(out + N, 2 * N * sizeof(double), W + (size_t)m * N, N * sizeof(double),
                             N * sizeof(double), m, hipMemcpyDeviceToDevice, c.stream));
    PPW_HIP(hipStreamSynchronize(c.stream));
    if (iters) *iters = it;
    if (worst) *worst = wr;
  });
}

pp_status ppint_products(pp_handle* h, int32_t order, int32_t k, const double* V, double* AV, double* BV, double* SV,
                         int32_t fp32) {
  if (!h || !h->ctx) return PP_EINVAL;
  return guarded(&h->err, [&] {
    settle(h);
    if (order < 0 || order > h->ctx->order) throw ppw::InvalidArg("order exceeds the setup order");
    if (fp32)
      ppw::sigma_core_f32(*h->ctx, order, k, V, AV, BV, SV);
    else
      ppw::sigma_core(*h->ctx, order, k, V, AV, BV, SV);
    PPW_HIP(hipStreamSynchronize(h->ctx->stream));
  });
}

}  // extern "C"
