// Helpers shared by the C entry points: exception -> status translation, input
// validation, option conversion.  Used only in the files that define extern "C"
// functions.
#pragma once

#include <cmath>
#include <string>

#include "../../include/ppwin.h"
#include "common.h"
#include "solver.h"

namespace ppw {

// Runs f and maps the library's exceptions to a status (message into *err).
template <typename F>
inline pp_status guarded(std::string* err, F&& f) {
  try {
    f();
    return PP_OK;
  } catch (const InvalidArg& e) {
    if (err) *err = e.what();
    return PP_EINVAL;
  } catch (const OutOfBudget& e) {
    if (err) *err = e.what();
    return PP_ENOMEM;
  } catch (const NotConverged& e) {
    if (err) *err = e.what();
    return PP_ENOTCONV;
  } catch (const Unstable& e) {
    if (err) *err = e.what();
    return PP_EUNSTABLE;
  } catch (const NotSupported& e) {
    if (err) *err = e.what();
    return PP_ENOTSUP;
  } catch (const DeviceError& e) {
    if (err) *err = e.what();
    return PP_EDEVICE;
  } catch (const std::exception& e) {
    if (err) *err = e.what();
    return PP_EDEVICE;
  } catch (...) {
    if (err) *err = "unknown error";
    return PP_EDEVICE;
  }
}

inline void check_finite(const double* p, size_t n, const char* what) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) throw InvalidArg(std::string("non-finite value in ") + what);
}

// Host-side checks of a system given by host pointers.
inline void check_host_system(const pp_system& sys) {
  const int o = sys.n_occ, v = sys.n_vir, X = sys.n_aux;
  const size_t N = (size_t)o * v;
  check_finite(sys.eps, (size_t)o + v, "eps");
  check_finite(sys.B_oo, (size_t)X * o * o, "B_oo");
  check_finite(sys.B_ov, (size_t)X * N, "B_ov");
  check_finite(sys.B_vv, (size_t)X * v * v, "B_vv");
  if (sys.dip) check_finite(sys.dip, 3 * N, "dip");
  for (int i = 0; i + 1 < o; ++i)
    if (sys.eps[i] > sys.eps[i + 1]) throw InvalidArg("occupied energies must be ascending");
  if (sys.eps[o - 1] >= sys.eps[o]) throw InvalidArg("occupied energies must lie below virtual ones");
}

inline void check_options(const pp_options& opt) {
  if (opt.precision != PP_FP64 && opt.precision != PP_FP32 && opt.precision != PP_SPLIT_BF16)
    throw InvalidArg("unknown precision");
  if (opt.max_basis > 512) throw InvalidArg("max_basis must be <= 512");
  if (!(opt.tol > 0)) throw InvalidArg("tol must be positive");
  if (opt.method != PP_FOLDED && opt.method != PP_RIESZ) throw InvalidArg("unknown method");
  if (opt.pass_vectors < 0) throw InvalidArg("pass_vectors must be >= 0");
  if (opt.method == PP_RIESZ) {
    if (opt.contour_nodes < 1 || opt.contour_nodes > 32) throw InvalidArg("contour_nodes must be in 1..32");
    if (!(opt.contour_tol > 0 && opt.contour_tol < 1)) throw InvalidArg("contour_tol must be in (0, 1)");
    if (opt.contour_maxit < 1) throw InvalidArg("contour_maxit must be positive");
  }
}

inline SolveOptions solve_options(const pp_options& o) {
  SolveOptions so;
  so.precision = o.precision == PP_FP64 ? 0 : 1;  // 1: reduced-precision products + FP64 refinement
  so.tol = o.tol;
  so.block = o.block;
  so.krylov_steps = o.krylov_steps;
  so.max_basis = o.max_basis;
  so.max_cycles = o.max_cycles;
  so.d_clamp = o.d_clamp;
  so.seed = o.seed;
  so.correlated_f = o.correlated_f;
  so.method = o.method;
  so.contour_nodes = o.contour_nodes;
  so.contour_tol = o.contour_tol;
  so.contour_maxit = o.contour_maxit;
  so.pass_vectors = o.pass_vectors;
  return so;
}

}  // namespace ppw
