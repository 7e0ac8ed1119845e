"""ctypes binding of libppwin (argument marshalling only).

Every computation happens in the HIP library; this module converts numpy arrays
and torch device tensors into the plain pointers and sizes of the C ABI declared
in include/ppwin.h and include/ppwin_testing.h.  Loading fails loudly when the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppwin.so")

PP_OK, PP_EINVAL, PP_ENOMEM, PP_ENOTCONV, PP_EUNSTABLE, PP_EDEVICE, PP_ENOTSUP, PP_EPENDING = range(8)
PP_FP64, PP_FP32, PP_SPLIT_BF16 = 0, 1, 2
PP_FOLDED, PP_RIESZ = 0, 1
PP_APPLY_METRIC = 1
PP_DEVICE_PTRS = 2
PP_ASYNC = 4
PP_REDUCED = 8
PP_MAX_ROOTS = 64


class PPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class pp_system(C.Structure):
    _fields_ = [("n_occ", C.c_int32), ("n_vir", C.c_int32), ("n_aux", C.c_int32), ("order", C.c_int32),
                ("eps", C.c_void_p), ("B_oo", C.c_void_p), ("B_ov", C.c_void_p), ("B_vv", C.c_void_p),
                ("dip", C.c_void_p), ("device_ptrs", C.c_int32)]


class pp_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("store_amplitudes", C.c_int32), ("strip_rows", C.c_int32),
                ("tol", C.c_double), ("block", C.c_int32), ("krylov_steps", C.c_int32),
                ("max_basis", C.c_int32), ("max_cycles", C.c_int32), ("d_clamp", C.c_double),
                ("hbm_budget", C.c_uint64), ("device", C.c_int32), ("stream", C.c_void_p),
                ("seed", C.c_uint64), ("tda", C.c_int32), ("correlated_f", C.c_int32),
                ("method", C.c_int32), ("contour_nodes", C.c_int32), ("contour_tol", C.c_double),
                ("contour_maxit", C.c_int32), ("pass_vectors", C.c_int32)]


class pp_solve_info(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("basis", C.c_int32), ("products", C.c_int64), ("n_roots", C.c_int32),
                ("converged", C.c_int32 * PP_MAX_ROOTS), ("residual", C.c_double * PP_MAX_ROOTS),
                ("seconds", C.c_double), ("sigma_seconds", C.c_double), ("sigma_flops", C.c_double)]


class pp_stats(C.Structure):
    _fields_ = [("product_flops", C.c_double), ("product_seconds", C.c_double), ("product_vectors", C.c_int64),
                ("hhat_flops", C.c_double), ("hhat_seconds", C.c_double), ("hhat_launches", C.c_int64)]


class ppint_gemm_member(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("K", C.c_int32), ("transA", C.c_int32), ("transB", C.c_int32),
                ("lda", C.c_int64), ("ldb", C.c_int64), ("ldc", C.c_int64), ("A", C.c_void_p), ("B", C.c_void_p),
                ("C", C.c_void_p), ("alpha", C.c_double), ("beta", C.c_double)]


class pp_result(C.Structure):
    _fields_ = [("energies", C.c_void_p), ("vectors", C.c_void_p), ("osc", C.c_void_p), ("n_roots", C.c_int32),
                ("status", C.c_int32), ("info", pp_solve_info), ("queued_seconds", C.c_double),
                ("run_seconds", C.c_double), ("latency_seconds", C.c_double)]


class pp_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("queued", C.c_int64),
                ("running", C.c_int64), ("peak_running", C.c_int32), ("latency_p50", C.c_double),
                ("latency_p99", C.c_double), ("queued_p50", C.c_double), ("queued_p99", C.c_double),
                ("solves_per_second", C.c_double), ("passes", C.c_int64), ("mean_requests_per_pass", C.c_double),
                ("product_flops", C.c_double), ("product_seconds", C.c_double), ("budget_bytes", C.c_uint64),
                ("reserved_bytes", C.c_uint64), ("peak_reserved_bytes", C.c_uint64), ("grouped_launches", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch (used by callers for device memory and streams) ships its own HIP and
        # HSA runtimes; they must initialize before the system runtime this library
        # links, or torch no longer finds the GPU.  Initialize torch's first when it is
        # installed (on a machine without a GPU this is a no-op).
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libppwin.so not found at {LIB_PATH}: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.pp_default_options.argtypes = [C.POINTER(pp_options)]
        L.pp_default_options.restype = None
        L.pp_setup.argtypes = [C.POINTER(pp_system), C.POINTER(pp_options), C.POINTER(vp)]
        L.pp_setup.restype = C.c_int
        L.pp_sigma.argtypes = [vp, i32, i32, vp, vp, u32]
        L.pp_sigma.restype = C.c_int
        L.pp_window_solve.argtypes = [vp, dbl, i32, vp, vp, vp, C.POINTER(pp_solve_info)]
        L.pp_window_solve.restype = C.c_int
        L.pp_window_solve_batch.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp]
        L.pp_window_solve_batch.restype = C.c_int
        L.pp_get_stats.argtypes = [vp, C.POINTER(pp_stats)]
        L.pp_get_stats.restype = C.c_int
        L.pp_reset_stats.argtypes = [vp]
        L.pp_reset_stats.restype = C.c_int
        L.pp_mp2_energy.argtypes = [vp]
        L.pp_mp2_energy.restype = dbl
        L.pp_device_bytes.argtypes = [vp]
        L.pp_device_bytes.restype = u64
        L.pp_sigma_static.argtypes = [vp, i32, i32, vp, vp, u32]
        L.pp_sigma_static.restype = C.c_int
        L.pp_sigma_part.argtypes = [vp, i32, i32, vp, vp, u32, i32, i32]
        L.pp_sigma_part.restype = C.c_int
        L.pp_sync.argtypes = [vp]
        L.pp_sync.restype = C.c_int
        L.pp_destroy.argtypes = [vp]
        L.pp_destroy.restype = C.c_int
        L.pp_status_string.argtypes = [C.c_int]
        L.pp_status_string.restype = C.c_char_p
        L.pp_last_error.argtypes = [vp]
        L.pp_last_error.restype = C.c_char_p
        L.ppint_gemm.argtypes = [i32, i32, i32, i32, i32, i32, i32, i64, i64, i64, i32, i64, i64, i64, i64, i64,
                                 dbl, vp, vp, dbl, vp, u64]
        L.ppint_gemm.restype = C.c_int
        L.ppint_gemm_cmap.argtypes = [i32, i32, i32, i32, i32, i64, i32, i64, i64, i32, i64, i32, i64, dbl, vp, vp,
                                      dbl, vp, C.c_uint64]
        L.ppint_gemm_cmap.restype = C.c_int
        L.ppint_inject_hip_error.argtypes = [i32, i32]
        L.ppint_inject_hip_error.restype = C.c_int
        L.ppint_split_sbf16.argtypes = [i64, vp]
        L.ppint_split_sbf16.restype = C.c_int
        L.ppint_gemm_group.argtypes = [i32, i32, C.POINTER(ppint_gemm_member), C.POINTER(i32)]
        L.ppint_gemm_group.restype = C.c_int
        L.ppint_partial_syev.argtypes = [i32, vp, dbl, i32, vp, vp, C.POINTER(i32)]
        L.ppint_partial_syev.restype = C.c_int
        L.ppint_syev.argtypes = [i32, vp, vp, vp]
        L.ppint_syev.restype = C.c_int
        L.ppint_cholesky.argtypes = [i32, vp, vp]
        L.ppint_cholesky.restype = C.c_int
        L.ppint_products.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32]
        L.ppint_products.restype = C.c_int
        L.ppint_riesz_filter.argtypes = [vp, dbl, dbl, i32, dbl, i32, i32, vp, vp, C.POINTER(i32), C.POINTER(dbl)]
        L.ppint_riesz_filter.restype = C.c_int
        L.pp_exciton_dos.argtypes = [vp, i32, vp, vp, vp]
        L.pp_exciton_dos.restype = C.c_int
        L.pp_response.argtypes = [i32, vp, vp, i32, vp, dbl, vp, vp]
        L.pp_response.restype = C.c_int
        L.pp_spectrum.argtypes = [i32, vp, vp, i32, vp, dbl, vp]
        L.pp_spectrum.restype = C.c_int
        L.pp_server_create.argtypes = [C.POINTER(pp_options), u64, i32, C.POINTER(vp)]
        L.pp_server_create.restype = C.c_int
        L.pp_server_submit.argtypes = [vp, C.POINTER(pp_system), dbl, i32, C.POINTER(u64)]
        L.pp_server_submit.restype = C.c_int
        L.pp_server_request_bytes.argtypes = [vp, C.POINTER(pp_system), i32]
        L.pp_server_request_bytes.restype = u64
        L.pp_server_poll.argtypes = [vp, u64, C.POINTER(pp_result)]
        L.pp_server_poll.restype = C.c_int
        L.pp_server_wait.argtypes = [vp, u64, C.POINTER(pp_result)]
        L.pp_server_wait.restype = C.c_int
        L.pp_server_stats_get.argtypes = [vp, C.POINTER(pp_server_stats)]
        L.pp_server_stats_get.restype = C.c_int
        L.pp_server_stats_reset.argtypes = [vp]
        L.pp_server_stats_reset.restype = C.c_int
        L.pp_server_destroy.argtypes = [vp]
        L.pp_server_destroy.restype = C.c_int
        L.pp_server_last_error.argtypes = [vp]
        L.pp_server_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st: int, handle=None):
    if st != PP_OK:
        L = lib()
        msg = L.pp_last_error(handle).decode() if handle is not None else L.pp_last_error(None).decode()
        raise PPError(st, f"{L.pp_status_string(st).decode()}: {msg}")


def default_options(**kw) -> pp_options:
    o = pp_options()
    lib().pp_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Handle:
    """A system set up on the device (wraps pp_handle*)."""

    def __init__(self, eps, B_oo, B_ov, B_vv, dip=None, order: int = 2, options: Optional[pp_options] = None,
                 device_ptrs: bool = False, **kw):
        L = lib()
        if device_ptrs:
            # torch device tensors (float64, contiguous), already resident in HBM
            arrs = [eps, B_oo, B_ov, B_vv] + ([dip] if dip is not None else [])
            for a in arrs:
                if not (a.is_cuda and a.is_contiguous()) or str(a.dtype) != "torch.float64":
                    raise ValueError("device inputs must be contiguous float64 device tensors")
            ptr = [a.data_ptr() for a in arrs]
            naux, o, v = B_ov.shape
        else:
            arrs = [_f64(eps), _f64(B_oo), _f64(B_ov), _f64(B_vv)] + ([_f64(dip)] if dip is not None else [])
            ptr = [a.ctypes.data for a in arrs]
            naux, o, v = arrs[2].shape
        self._arrays = arrs
        s = pp_system(n_occ=o, n_vir=v, n_aux=naux, order=order, eps=ptr[0], B_oo=ptr[1], B_ov=ptr[2],
                      B_vv=ptr[3], dip=ptr[4] if dip is not None else None, device_ptrs=1 if device_ptrs else 0)
        opt = options if options is not None else default_options(**kw)
        h = C.c_void_p()
        st = L.pp_setup(C.byref(s), C.byref(opt), C.byref(h))
        self._arrays = None
        _check(st)
        self.h = h
        self.o, self.v, self.naux, self.order = o, v, naux, order
        self.N = o * v

    @classmethod
    def from_system(cls, sys, order: int = 2, **kw):
        return cls(sys.eps, sys.B_oo, sys.B_ov, sys.B_vv, sys.dip, order=order, **kw)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().pp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def sigma(self, X, order: Optional[int] = None, metric: bool = False, reduced: bool = False) -> np.ndarray:
        """M X (or Sigma X) for host X of shape [m][2][o][v] or [m][2][N]; reduced=True runs
        the contractions in the handle's reduced precision (PP_REDUCED)."""
        X = _f64(X)
        m = X.shape[0]
        out = np.empty((m, 2, self.N))
        flags = (PP_APPLY_METRIC if metric else 0) | (PP_REDUCED if reduced else 0)
        st = lib().pp_sigma(self.h, self.order if order is None else order, m, X.ctypes.data, out.ctypes.data, flags)
        _check(st, self.h)
        return out

    def sigma_device(self, X, out, order: Optional[int] = None, metric: bool = False, async_: bool = False,
                     reduced: bool = False):
        """Same as sigma() on torch device tensors (no host copies).  async_=True returns
        once the product is enqueued on the handle's stream (see sync())."""
        m = X.shape[0]
        flags = (PP_DEVICE_PTRS | (PP_APPLY_METRIC if metric else 0) | (PP_ASYNC if async_ else 0)
                 | (PP_REDUCED if reduced else 0))
        st = lib().pp_sigma(self.h, self.order if order is None else order, m, X.data_ptr(), out.data_ptr(), flags)
        _check(st, self.h)

    def sigma_static(self, X, out, order: Optional[int] = None, metric: bool = False, reduced: bool = False):
        """pp_sigma_static on torch device tensors [m][2][N]: the product with no allocation
        (staging in the library's fixed scratch array)."""
        m = X.shape[0]
        flags = PP_DEVICE_PTRS | (PP_APPLY_METRIC if metric else 0) | (PP_REDUCED if reduced else 0)
        st = lib().pp_sigma_static(self.h, self.order if order is None else order, m, X.data_ptr(),
                                   out.data_ptr(), flags)
        _check(st, self.h)

    def sigma_part(self, X, out, part: int, n_parts: int, order: Optional[int] = None, metric: bool = False,
                   reduced: bool = False, async_: bool = False):
        """One part of a product pass issued in parts (pp_sigma_part).  X, out: torch device
        tensors [m][2][N] (device pointers) or numpy arrays (host pointers, out filled after
        the last part)."""
        dev = hasattr(X, "data_ptr")
        m = X.shape[0]
        flags = ((PP_DEVICE_PTRS if dev else 0) | (PP_APPLY_METRIC if metric else 0) | (PP_ASYNC if async_ else 0)
                 | (PP_REDUCED if reduced else 0))
        xp = X.data_ptr() if dev else X.ctypes.data
        op = out.data_ptr() if dev else out.ctypes.data
        st = lib().pp_sigma_part(self.h, self.order if order is None else order, m, xp, op, flags, int(part),
                                 int(n_parts))
        _check(st, self.h)

    def sync(self):
        """Waits for the products enqueued with async_=True."""
        _check(lib().pp_sync(self.h), self.h)

    def products(self, V, AV, BV, SV=None, order: Optional[int] = None, fp32: bool = False):
        """A V, B V, S V for torch device tensors [k][N] (internal test hook)."""
        st = lib().ppint_products(self.h, self.order if order is None else order, V.shape[0], V.data_ptr(),
                                  AV.data_ptr(), BV.data_ptr(), SV.data_ptr() if SV is not None else None,
                                  1 if fp32 else 0)
        _check(st, self.h)

    def riesz_filter(self, V, out, center: float, radius: float, nodes: int, tol: float = 1e-10,
                     maxit: int = 500):
        """out = P V for torch device tensors [m][2][N] (contour quadrature of the resolvent;
        internal test hook).  Returns (largest iteration count, largest final relative
        residual) of the shifted solves."""
        it, worst = C.c_int32(0), C.c_double(0.0)
        st = lib().ppint_riesz_filter(self.h, float(center), float(radius), int(nodes), float(tol), int(maxit),
                                      V.shape[0], V.data_ptr(), out.data_ptr(), C.byref(it), C.byref(worst))
        _check(st, self.h)
        return it.value, worst.value

    def window_solve(self, omega0: float, n_roots: int, vectors: bool = True, osc: bool = True,
                     allow_unconverged: bool = False):
        """Returns (energies, vectors [r][2][N] or None, osc or None, info dict)."""
        e = np.empty(n_roots)
        vec = np.empty((n_roots, 2, self.N)) if vectors else None
        f = np.empty(n_roots) if osc else None
        info = pp_solve_info()
        st = lib().pp_window_solve(self.h, float(omega0), n_roots, e.ctypes.data,
                                   vec.ctypes.data if vec is not None else None,
                                   f.ctypes.data if f is not None else None, C.byref(info))
        if not (st == PP_ENOTCONV and allow_unconverged):
            _check(st, self.h)
        d = dict(cycles=info.cycles, basis=info.basis, products=info.products, seconds=info.seconds,
                 sigma_seconds=info.sigma_seconds, sigma_flops=info.sigma_flops,
                 residual=np.array(info.residual[:n_roots]), converged=np.array(info.converged[:n_roots]),
                 status=st)
        return e, vec, f, d

    def stats(self) -> dict:
        st = pp_stats()
        _check(lib().pp_get_stats(self.h, C.byref(st)), self.h)
        return dict(product_flops=st.product_flops, product_seconds=st.product_seconds,
                    product_vectors=st.product_vectors, hhat_flops=st.hhat_flops, hhat_seconds=st.hhat_seconds,
                    hhat_launches=st.hhat_launches)

    def reset_stats(self):
        _check(lib().pp_reset_stats(self.h), self.h)

    def window_solve_batch(self, omegas, n_roots: int, vectors: bool = True, osc: bool = True,
                           allow_unconverged: bool = False):
        """All windows in one call; returns (energies [w][r], vectors [w][r][2][N] or None,
        osc [w][r] or None, list of info dicts)."""
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        nw = len(om)
        e = np.empty((nw, n_roots))
        vec = np.empty((nw, n_roots, 2, self.N)) if vectors else None
        f = np.empty((nw, n_roots)) if osc else None
        infos = (pp_solve_info * nw)()
        st = lib().pp_window_solve_batch(self.h, nw, om.ctypes.data, n_roots, e.ctypes.data,
                                         vec.ctypes.data if vec is not None else None,
                                         f.ctypes.data if f is not None else None, infos)
        if not (st == PP_ENOTCONV and allow_unconverged):
            _check(st, self.h)
        out = []
        for w in range(nw):
            info = infos[w]
            out.append(dict(cycles=info.cycles, basis=info.basis, products=info.products, seconds=info.seconds,
                            sigma_seconds=info.sigma_seconds, sigma_flops=info.sigma_flops,
                            residual=np.array(info.residual[:n_roots]),
                            converged=np.array(info.converged[:n_roots]), status=st))
        return e, vec, f, out

    def exciton_dos(self, edges):
        """(counts, mu2) per energy bin of the particle-hole energies eps_a - eps_i."""
        ed = _f64(edges).ravel()
        nb = len(ed) - 1
        counts, mu2 = np.empty(nb), np.empty(nb)
        _check(lib().pp_exciton_dos(self.h, nb, ed.ctypes.data, counts.ctypes.data, mu2.ctypes.data), self.h)
        return counts, mu2

    def mp2_energy(self) -> float:
        return lib().pp_mp2_energy(self.h)

    def device_bytes(self) -> int:
        return int(lib().pp_device_bytes(self.h))


def gemm(A, B, C_, *, M, N, K, KB=1, nbatch=1, transA=0, lda, sA=0, sAk=0, transB=0, ldb, sB=0, sBk=0, ldc,
         sC=0, alpha=1.0, beta=0.0, ws_bytes=0, fp32=False):
    """Library GEMM on torch device tensors (internal test hook)."""
    st = lib().ppint_gemm(int(fp32), M, N, K, KB, nbatch, transA, lda, sA, sAk, transB, ldb, sB, sBk, ldc, sC,
                          alpha, A.data_ptr(), B.data_ptr(), beta, C_.data_ptr(), ws_bytes)
    _check(st)


def gemm_cmap(A, B, C_, *, M, N, K, transA=0, lda, transB=0, ldb, ldc, cRm=0, cSm=0, cRn=0, cSn=0, alpha=1.0,
              beta=0.0, ws_bytes=0, fp32=False):
    """Library GEMM with C rows/columns split into index pairs (internal test hook)."""
    st = lib().ppint_gemm_cmap(int(fp32), M, N, K, transA, lda, transB, ldb, ldc, cRm, cSm, cRn, cSn, alpha,
                               A.data_ptr(), B.data_ptr(), beta, C_.data_ptr(), ws_bytes)
    _check(st)


def inject_hip_error(after_calls: int, code: int = 0):
    """Failure injection (test hook): the after_calls-th checked HIP call reports 'code'."""
    _check(lib().ppint_inject_hip_error(int(after_calls), int(code)))


def split_sbf16(x):
    """In-place split of a float32 device tensor into the split-BF16 chunk layout (test hook)."""
    _check(lib().ppint_split_sbf16(x.numel(), x.data_ptr()))


def gemm_group(members, fp32=False) -> int:
    """Grouped GEMM test hook: members are dicts with torch device tensors A, B, C and
    M, N, K, transA, transB, lda, ldb, ldc, alpha, beta.  Returns the grouped launch count."""
    arr = (ppint_gemm_member * len(members))()
    for i, m in enumerate(members):
        arr[i] = ppint_gemm_member(M=m["M"], N=m["N"], K=m["K"], transA=m["transA"], transB=m["transB"],
                                   lda=m["lda"], ldb=m["ldb"], ldc=m["ldc"], A=m["A"].data_ptr(),
                                   B=m["B"].data_ptr(), C=m["C"].data_ptr(), alpha=m.get("alpha", 1.0),
                                   beta=m.get("beta", 0.0))
    g = C.c_int32()
    _check(lib().ppint_gemm_group(1 if fp32 else 0, len(members), arr, C.byref(g)))
    return g.value


def partial_syev(A, target, p, lam, Z) -> int:
    q = C.c_int32()
    _check(lib().ppint_partial_syev(A.shape[0], A.data_ptr(), float(target), int(p), lam.data_ptr(), Z.data_ptr(),
                                    C.byref(q)))
    return q.value


def syev(A, w, Z):
    _check(lib().ppint_syev(A.shape[0], A.data_ptr(), w.data_ptr(), Z.data_ptr()))


def cholesky(A, L_):
    _check(lib().ppint_cholesky(A.shape[0], A.data_ptr(), L_.data_ptr()))


def spectrum(energies, osc, omega, eta: float) -> np.ndarray:
    """Lorentzian-broadened oscillator-strength spectrum on the grid omega (pp_spectrum)."""
    e, f, w = _f64(energies).ravel(), _f64(osc).ravel(), _f64(omega).ravel()
    if e.shape != f.shape:
        raise ValueError("energies and osc must have the same length")
    out = np.empty_like(w)
    _check(lib().pp_spectrum(len(e), e.ctypes.data, f.ctypes.data, len(w), w.ctypes.data, float(eta),
                             out.ctypes.data))
    return out


def response(energies, osc, omega, eta: float) -> np.ndarray:
    """The isotropic dipole propagator Pi(omega + i eta) assembled from roots (pp_response),
    as a complex array over the grid omega."""
    e, f, w = _f64(energies).ravel(), _f64(osc).ravel(), _f64(omega).ravel()
    if e.shape != f.shape:
        raise ValueError("energies and osc must have the same length")
    re, im = np.empty_like(w), np.empty_like(w)
    _check(lib().pp_response(len(e), e.ctypes.data, f.ctypes.data, len(w), w.ctypes.data, float(eta),
                             re.ctypes.data, im.ctypes.data))
    return re + 1j * im


class Server:
    """The serving loop (wraps pp_server*): submit window solves of differing systems,
    collect results; requests solving together share merged product passes."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 0, **opts):
        L = lib()
        o = default_options(**opts)
        h = C.c_void_p()
        st = L.pp_server_create(C.byref(o), hbm_budget, max_active, C.byref(h))
        if st != PP_OK:
            raise PPError(st, f"{L.pp_status_string(st).decode()}: {L.pp_server_last_error(None).decode()}")
        self.h = h
        self._meta = {}

    def _check(self, st):
        if st != PP_OK:
            L = lib()
            raise PPError(st, f"{L.pp_status_string(st).decode()}: {L.pp_server_last_error(self.h).decode()}")

    def submit(self, eps, B_oo, B_ov, B_vv, dip, omega0: float, n_roots: int, order: int = 2) -> int:
        arrs = [_f64(eps), _f64(B_oo), _f64(B_ov), _f64(B_vv)] + ([_f64(dip)] if dip is not None else [])
        naux, o, v = arrs[2].shape
        s = pp_system(n_occ=o, n_vir=v, n_aux=naux, order=order, eps=arrs[0].ctypes.data,
                      B_oo=arrs[1].ctypes.data, B_ov=arrs[2].ctypes.data, B_vv=arrs[3].ctypes.data,
                      dip=arrs[4].ctypes.data if dip is not None else None, device_ptrs=0)
        rid = C.c_uint64()
        self._check(lib().pp_server_submit(self.h, C.byref(s), float(omega0), int(n_roots), C.byref(rid)))
        self._meta[rid.value] = (o * v, int(n_roots))
        return rid.value

    def request_bytes(self, o: int, v: int, naux: int, n_roots: int, order: int = 2, dip: bool = True) -> int:
        dummy = np.zeros(1)
        s = pp_system(n_occ=o, n_vir=v, n_aux=naux, order=order, eps=dummy.ctypes.data, B_oo=dummy.ctypes.data,
                      B_ov=dummy.ctypes.data, B_vv=dummy.ctypes.data, dip=dummy.ctypes.data if dip else None,
                      device_ptrs=0)
        return int(lib().pp_server_request_bytes(self.h, C.byref(s), int(n_roots)))

    def submit_system(self, sys, omega0: float, n_roots: int, order: int = 2) -> int:
        return self.submit(sys.eps, sys.B_oo, sys.B_ov, sys.B_vv, sys.dip, omega0, n_roots, order)

    def _take(self, rid: int, block: bool, allow_unconverged: bool):
        N, nr = self._meta[rid]
        e = np.zeros(nr)
        vec = np.zeros((nr, 2, N))
        f = np.zeros(nr)
        res = pp_result(energies=e.ctypes.data, vectors=vec.ctypes.data, osc=f.ctypes.data)
        fn = lib().pp_server_wait if block else lib().pp_server_poll
        st = fn(self.h, rid, C.byref(res))
        if st == PP_EPENDING:
            return None
        del self._meta[rid]
        if not (st == PP_OK or (st == PP_ENOTCONV and allow_unconverged)):
            self._check(st)
        info = res.info
        return dict(energies=e, vectors=vec, osc=f, status=st, n_roots=res.n_roots,
                    queued_seconds=res.queued_seconds, run_seconds=res.run_seconds,
                    latency_seconds=res.latency_seconds, products=info.products, cycles=info.cycles,
                    residual=np.array(info.residual[:nr]), converged=np.array(info.converged[:nr]))

    def wait(self, rid: int, allow_unconverged: bool = False):
        return self._take(rid, True, allow_unconverged)

    def poll(self, rid: int, allow_unconverged: bool = False):
        return self._take(rid, False, allow_unconverged)

    def stats(self) -> dict:
        st = pp_server_stats()
        self._check(lib().pp_server_stats_get(self.h, C.byref(st)))
        return {name: getattr(st, name) for name, _ in pp_server_stats._fields_}

    def reset_stats(self):
        self._check(lib().pp_server_stats_reset(self.h))

    def close(self):
        if self.h:
            lib().pp_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
