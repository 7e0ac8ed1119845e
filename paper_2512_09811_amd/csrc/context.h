// Device-resident state of one system (the object behind a pp_handle).
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace ppw {

// Row stride, in values, of FP32 / split-BF16 rows of n values: n rounded up to whole
// 8-value chunks, plus 64 values (256 B) when that would start the rows a multiple of
// 4 KiB apart.  Rows 1 MiB apart (n = 262144) all start on the same memory channels and
// a 256-row GEMM tile of them ran 6% slower than with the 256 B offset.
inline long padded_stride(long n) {
  const long p = (n + 7) / 8 * 8;
  return (p * 4) % 4096 == 0 ? p + 64 : p;
}

// Device allocations with a byte budget.  Every allocation of a handle goes
// through its arena, so the footprint is known and bounded.
class Arena {
 public:
  explicit Arena(size_t budget = 0) : budget_(budget) {}
  ~Arena() { release(); }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;

  void set_budget(size_t b) { budget_ = b; }
  size_t used() const { return used_; }
  size_t budget() const { return budget_; }

  template <typename T>
  T* alloc(size_t n, const char* what) {
    const size_t bytes = ((n * sizeof(T) + 255) / 256) * 256;
    if (budget_ && used_ + bytes > budget_)
      throw OutOfBudget(std::string("device budget exceeded allocating ") + what + " (" +
                        std::to_string(bytes) + " B, " + std::to_string(used_) + " of " +
                        std::to_string(budget_) + " B in use)");
    void* p = nullptr;
    if (bytes) {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw OutOfBudget(std::string("hipMalloc failed for ") + what + ": " + hipGetErrorString(e));
      }
    }
    blocks_.push_back({p, bytes});
    used_ += bytes;
    return static_cast<T*>(p);
  }
  void free(void* p) {
    for (size_t i = 0; i < blocks_.size(); ++i)
      if (blocks_[i].p == p) {
        if (p) (void)hipFree(p);
        used_ -= blocks_[i].bytes;
        blocks_.erase(blocks_.begin() + i);
        return;
      }
  }
  void release() {
    for (auto& b : blocks_)
      if (b.p) (void)hipFree(b.p);
    blocks_.clear();
    used_ = 0;
  }

 private:
  struct Block {
    void* p;
    size_t bytes;
  };
  std::vector<Block> blocks_;
  size_t used_ = 0;
  size_t budget_ = 0;
};

struct SetupParams {
  int o = 0, v = 0, naux = 0, order = 1;
  const double *eps = nullptr, *Boo = nullptr, *Bov = nullptr, *Bvv = nullptr, *dip = nullptr;
  bool device_ptrs = false;
  int store_amplitudes = -1;  // -1 auto
  int strip_rows = 0;
  bool want_f32 = false;       // keep FP32 copies for the reduced-precision product path
  bool split_bf16 = false;     // reduced-precision amplitude contraction as split-BF16 products
  bool tda = false;            // Tamm-Dancoff: B = 0
  size_t budget = 0;
  int device = 0;
  hipStream_t stream = nullptr;
};

// Timing/flop accounting of product passes.
struct SigmaStats {
  double flops = 0.0;       // algorithmic flops issued by product passes
  double flops32 = 0.0;     // of which on the FP32 path
  double seconds = 0.0;     // device time of product passes (events)
  long vectors = 0;         // particle-hole vectors multiplied
  double hhat_flops = 0.0;  // flops of the amplitude-weighted contraction (dominant kernel)
  double hhat_seconds = 0.0;
  long hhat_launches = 0;
};

// HIP events recorded around product passes and around the dominant GEMM, kept
// unresolved (no host synchronization in the hot path) until stats are read.
class EventLog {
 public:
  ~EventLog() {
    for (auto& r : recs_) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool_) (void)hipEventDestroy(e);
  }
  int start(hipStream_t s) {
    Rec r{get(), get(), -1, 0.0};
    PPW_HIP(hipEventRecord(r.a, s));
    recs_.push_back(r);
    return (int)recs_.size() - 1;
  }
  void stop(int i, hipStream_t s, int kind) {
    recs_[i].kind = kind;
    PPW_HIP(hipEventRecord(recs_[i].b, s));
  }
  // synchronizes on the recorded events and adds elapsed seconds per kind
  // (records whose stop was never reached, after an error, are discarded)
  void resolve(double* seconds_by_kind, int nkinds) {
    for (auto& r : recs_) {
      if (r.kind >= 0 && r.kind < nkinds) {
        PPW_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        PPW_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        seconds_by_kind[r.kind] += 1e-3 * ms;
      }
      pool_.push_back(r.a);
      pool_.push_back(r.b);
    }
    recs_.clear();
  }
  size_t pending() const { return recs_.size(); }

 private:
  struct Rec {
    hipEvent_t a, b;
    int kind;
    double flops;
  };
  hipEvent_t get() {
    if (!pool_.empty()) {
      hipEvent_t e = pool_.back();
      pool_.pop_back();
      return e;
    }
    hipEvent_t e;
    PPW_HIP(hipEventCreate(&e));
    return e;
  }
  std::vector<Rec> recs_;
  std::vector<hipEvent_t> pool_;
};

struct Context {
  int o = 0, v = 0, naux = 0, order = 0;
  long N = 0;
  long N8 = 0;  // row stride of the FP32 / split-BF16 G and amplitude rows (padded_stride(N))
  int X8 = 0;   // naux rounded up to a multiple of 8
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Arena arena;

  // inputs (device)
  double *eps_o = nullptr, *eps_v = nullptr;
  double *Bov = nullptr, *Boo = nullptr, *Bvv = nullptr, *dip = nullptr;
  // correlated property vector S mu (order 2 with dipoles; equals dip below order 2)
  double* dipS = nullptr;
  // derived layouts
  double* BovLam = nullptr;  // [ns][naux][N]: Bov, then Lambda at order 2
  double* Lam = nullptr;     // Lambda_P,ia = sum_kc tau_ik^ac B_P,kc
  double* Boo_t = nullptr;   // [o][o][naux]
  double* R = nullptr;       // [o][ns][naux][v] ring operand
  int ns = 1;
  // second-order intermediates
  double *Gv = nullptr, *Ev = nullptr, *Go = nullptr, *Eo = nullptr;
  // diagonals of A, B (first order part) and S
  double *dA = nullptr, *dB = nullptr, *dS = nullptr;
  // stored amplitudes tau[(i,c)][(j,d)] (optional)
  double* tau = nullptr;
  int strip_rows = 0;
  double emp2 = 0.0;
  bool tda = false;  // Tamm-Dancoff: every B product (and the B diagonal) is zero
  bool split_bf16 = false;  // reduced-precision amplitude contraction on BF16 matrix cores

  // FP32 copies for the reduced-precision path (optional)
  float *Bov32 = nullptr, *Boo32 = nullptr, *Bvv32 = nullptr, *BovLam32 = nullptr, *Boo_t32 = nullptr,
        *R32 = nullptr, *tau32 = nullptr;
  float *Gv32 = nullptr, *Ev32 = nullptr, *Go32 = nullptr, *Eo32 = nullptr;
  // split-BF16 operands (split layout of split_sbf16): stored amplitudes [N][N8] and,
  // for amplitudes rebuilt in strips, B^ov transposed [N][X8]
  float *tau_sbf = nullptr, *BovT_sbf = nullptr;

  // product workspace (grown on demand)
  int kcap = 0;
  int kcap32 = 0;
  int kcap_asm = 0;
  double *w_c = nullptr, *w_J = nullptr, *w_G = nullptr, *w_U = nullptr, *w_H = nullptr, *w_S = nullptr,
         *w_tau = nullptr, *w_P = nullptr;
  float *w32_V = nullptr, *w32_c = nullptr, *w32_J = nullptr, *w32_G = nullptr, *w32_U = nullptr,
        *w32_H = nullptr, *w32_S = nullptr, *w32_tau = nullptr, *w32_P = nullptr, *w32_AV = nullptr,
        *w32_BV = nullptr;
  Workspace ws;      // split-K workspace
  size_t ws_bytes = 0;

  SigmaStats stats;
  EventLog events;
  long pass_serial = 0;  // product passes started on this context (a part sequence checks it)
  bool no_events = false;  // products record no timing events (and create none)
  std::string last_error;

  // folds pending event timings into stats (synchronizes on them)
  void resolve_stats() {
    double sec[2] = {0.0, 0.0};
    events.resolve(sec, 2);
    stats.seconds += sec[0];
    stats.hhat_seconds += sec[1];
  }

  ~Context();
};

// Builds a context (copies inputs, layouts, diagonals, MP2 intermediates).
Context* setup_context(const SetupParams& p);

// Part of a product pass: pre runs every contraction that does not depend on the
// amplitude strips (with stored amplitudes, the amplitude contraction too), rows
// [i0, i1) (i1 < 0: to n_occ) the strips of those occupied rows, post the final FP64
// combination.  The parts of one pass cover the occupied rows once, pre first and post
// last, with no other product on the context in between (they share its workspaces).
struct PassRange {
  bool pre = true;
  int i0 = 0, i1 = -1;
  bool post = true;
};

// Products of k particle-hole vectors V ([k][o][v], device): AV = A V, BV = B V,
// SV = S V (SV may be null) at the given order (<= ctx order).  Device pointers.
void sigma_core(Context& c, int order, int k, const double* V, double* AV, double* BV, double* SV);

// Same products with the contractions on FP32 matrix cores (V and outputs FP64).
void sigma_core_f32(Context& c, int order, int k, const double* V, double* AV, double* BV, double* SV);

// One part of a product pass (prec 0: FP64 contractions; 1: the context's reduced
// precision, FP32 or split-BF16 amplitude products) on the context's stream.
void sigma_pass(Context& c, int order, int k, int prec, const double* V, double* AV, double* BV, double* SV,
                const PassRange& rg);

// One system's share of a merged product pass.
struct PassJob {
  Context* c = nullptr;
  int order = 0;
  int k = 0;
  int prec = 0;  // 0: FP64 contractions, 1: FP32 contractions (FP64 assembly)
  const double* V = nullptr;
  double *AV = nullptr, *BV = nullptr, *SV = nullptr;
};

// Products of several systems (distinct contexts) in one pass on stream s: every
// contraction step is issued for all systems together, its GEMMs merged into grouped
// launches.  No GEMM takes split-K unless its split was fixed when it was recorded, so a
// system's products are bitwise the same whichever systems share the pass.  Each context's workspace must already hold its k vectors
// (sigma_reserve); inputs must be ready on s.  Returns the number of grouped GEMM
// launches issued (steps whose GEMMs were too small to fill the chip together are
// launched one by one).
int sigma_group(const std::vector<PassJob>& jobs, hipStream_t s);

// Device bytes of a context for the given shape and policy: during setup (amplitude
// strips included) and afterwards with product workspaces for k vectors (FP64, plus
// FP32 when want_f32).  Upper bounds of what setup_context and sigma_reserve allocate.
struct Footprint {
  size_t setup_peak, steady;
};
Footprint context_footprint(int o, int v, int naux, int order, bool dip, bool store, int strip_rows, bool want_f32,
                            int k, bool split = false);

// Whether the product workspace already holds k vectors at that order and precision,
// so that a pass allocates nothing.
bool sigma_workspace_ready(const Context& c, int order, int k, int prec);

// Grows the product workspace to k vectors ahead of time (no allocation in the loop).
void sigma_reserve(Context& c, int k, int precision);
// Device bytes that sigma_reserve(c, k, precision) would add to the context's arena.
size_t sigma_reserve_bytes(const Context& c, int k, int precision);

// Algorithmic flops of one product pass over k vectors at the given order, with the
// contractions of precision prec (0 FP64, 1 reduced); amplitudes that precision does not
// store are rebuilt in strips, and their integrals count.
double sigma_flops(const Context& c, int order, int k, int prec = 0);

}  // namespace ppw
