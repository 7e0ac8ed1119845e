"""Parity of the HIP path against the FP64 oracle, through the C ABI.

Products (pp_sigma) at orders 0-2 are compared element by element with the
dense oracle on seeded systems that span several GEMM tiles and ragged tails;
window solves are compared root by root with the oracle's exact pencil
solution.  Tolerances: products 1e-12 relative to the largest element (FP64
throughout); energies 1e-8 Ha (the target accuracy is 1e-6 Ha; the FP64 solver
converges residuals to 1e-9); oscillator strengths 1e-5 relative above
1e-4 max(f), 1e-9 absolute below.
"""
import numpy as np
import pytest

from synth import gen
from synth.gen import random_block
from oracle import dense, pencil

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2512_09811_amd as P
    P.lib()
    return P


SYSTEMS = {
    "c1": dict(seed=1, o=8, v=24, naux=64),
    "mid": dict(seed=7, o=12, v=40, naux=100, b_scale=0.3),
    "ragged": dict(seed=11, o=5, v=19, naux=23, b_scale=0.5),
    # N = 1024: FP32 rows of N values would start 4 KiB apart, so their stride is padded
    "pad": dict(seed=13, o=16, v=64, naux=40, b_scale=0.3),
}


def _sys(name):
    p = dict(SYSTEMS[name])
    return gen(p.pop("seed"), p.pop("o"), p.pop("v"), p.pop("naux"), **p)


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("store", [1, 0])
def test_sigma_matches_dense_oracle(P, name, store):
    sys = _sys(name)
    print(f"[sigma parity] system={name} store={store} o={sys.o} v={sys.v} naux={sys.naux}", flush=True)
    X = random_block(5, sys.N, 3)
    with P.Handle.from_system(sys, order=2, store_amplitudes=store, strip_rows=3) as h:
        got = {k: h.sigma(X, order=k) for k in (0, 1, 2)}
        gotS = h.sigma(X, order=2, metric=True)
        e2 = h.mp2_energy()
    ref = {k: dense.sigma_dense(sys, k, X) for k in (0, 1, 2)}
    refS = dense.sigma_dense(sys, 2, X, metric=True)
    scale = np.abs(ref[2]).max()
    for k in (0, 1, 2):
        np.testing.assert_allclose(got[k], ref[k], rtol=0, atol=1e-12 * scale)
    # the second-order part on its own (small next to the zeroth-order diagonal)
    d_ref = ref[2] - ref[1]
    d_got = got[2] - got[1]
    assert np.abs(d_ref).max() > 1e-6 * scale
    np.testing.assert_allclose(d_got, d_ref, rtol=0, atol=1e-10 * np.abs(d_ref).max())
    np.testing.assert_allclose(gotS, refS, rtol=0, atol=1e-13)
    assert abs(e2 - dense.mp2_energy(sys)) < 1e-12 * abs(dense.mp2_energy(sys))


def test_sigma_order1_handle(P):
    sys = _sys("ragged")
    X = random_block(9, sys.N, 2)
    with P.Handle.from_system(sys, order=1) as h:
        got = h.sigma(X)
    np.testing.assert_allclose(got, dense.sigma_dense(sys, 1, X), rtol=0, atol=1e-13)


def test_sigma_async(P):
    """PP_ASYNC products against the oracle: on the caller's stream they are read in
    stream order (two calls in a row, the second larger so the handle's staging grows);
    on the handle's own stream they are settled by sync() or by the next call on the
    handle; host pointers are refused."""
    import torch
    sys = _sys("mid")
    X, X2 = random_block(5, sys.N, 4), random_block(6, sys.N, 7)
    ref, ref2 = dense.sigma_dense(sys, 2, X), dense.sigma_dense(sys, 2, X2)
    tol = 1e-12 * max(np.abs(ref).max(), np.abs(ref2).max())
    s = torch.cuda.Stream()
    with P.Handle.from_system(sys, order=2, stream=s.cuda_stream) as h:
        with torch.cuda.stream(s):
            dX, dX2 = torch.tensor(X, device="cuda"), torch.tensor(X2, device="cuda")
            out, out2 = torch.empty_like(dX), torch.empty_like(dX2)
            h.sigma_device(dX, out, async_=True)
            h.sigma_device(dX2, out2, async_=True)
            got, got2 = out.cpu().numpy(), out2.cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=0, atol=tol)
        np.testing.assert_allclose(got2, ref2, rtol=0, atol=tol)
    with P.Handle.from_system(sys, order=2) as h:
        dX = torch.tensor(X, device="cuda")
        torch.cuda.synchronize()
        out, out2 = torch.empty_like(dX), torch.empty_like(dX)
        h.sigma_device(dX, out, async_=True)
        h.sync()
        np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=0, atol=tol)
        h.sigma_device(dX, out2, async_=True)
        host = h.sigma(X)  # a synchronous call waits for the pending product first
        np.testing.assert_allclose(out2.cpu().numpy(), ref, rtol=0, atol=tol)
        np.testing.assert_allclose(host, ref, rtol=0, atol=tol)
        hout = np.empty_like(X)
        st = P.lib().pp_sigma(h.h, 2, X.shape[0], X.ctypes.data, hout.ctypes.data, P.PP_ASYNC)
        assert st == P.PP_EINVAL


def _check_window(sys, order, omega0, nr, e, vec, f, info):
    A, B, S = dense.assemble(sys, order)
    e_ref, X_ref, Y_ref, f_ref = pencil.window_solve(A, B, S, sys.dip, omega0, nr)
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-8)
    big = f_ref >= 1e-4 * f_ref.max()
    np.testing.assert_allclose(f[big], f_ref[big], rtol=1e-5)
    np.testing.assert_allclose(f[~big], f_ref[~big], rtol=0, atol=1e-9)
    # eigenvectors: unique up to sign for non-degenerate roots; S-normalized
    for q in range(nr):
        x, y = vec[q, 0], vec[q, 1]
        nrm = x @ S @ x - y @ S @ y
        assert abs(nrm - 1.0) < 1e-8
        ov = abs(x @ S @ X_ref[:, q] - y @ S @ Y_ref[:, q])
        assert abs(ov - 1.0) < 1e-6
    assert np.all(info["converged"] == 1)


@pytest.mark.parametrize("order", [1, 2])
def test_window_c1(P, order):
    sys = gen(1, 8, 24, 64)
    print(f"[window] rpa o=8 v=24 naux=64 order={order}", flush=True)
    with P.Handle.from_system(sys, order=order) as h:
        e, vec, f, info = h.window_solve(0.5, 6)
    _check_window(sys, order, 0.5, 6, e, vec, f, info)


@pytest.mark.parametrize("omega0,nr", [(0.45, 8), (1.1, 8), (1.6, 5)])
def test_window_mid(P, omega0, nr):
    sys = gen(7, 12, 40, 100)
    print(f"[window] mid o=12 v=40 naux=100 omega0={omega0}", flush=True)
    with P.Handle.from_system(sys, order=2) as h:
        e, vec, f, info = h.window_solve(omega0, nr)
    _check_window(sys, 2, omega0, nr, e, vec, f, info)


def test_window_deterministic(P):
    sys = gen(7, 12, 40, 100)
    with P.Handle.from_system(sys, order=2) as h:
        a = h.window_solve(0.8, 6)
        b = h.window_solve(0.8, 6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_error_paths(P):
    sys = gen(1, 8, 24, 64)
    bad = gen(1, 8, 24, 64)
    bad.B_ov[0, 0, 0] = np.nan
    with pytest.raises(P.PPError) as ei:
        P.Handle.from_system(bad)
    assert ei.value.status == P.PP_EINVAL
    with pytest.raises(P.PPError) as ei:
        P.Handle.from_system(sys, hbm_budget=1 << 16)
    assert ei.value.status == P.PP_ENOMEM
    with P.Handle.from_system(sys, order=1) as h:
        with pytest.raises(P.PPError) as ei:
            h.sigma(random_block(1, sys.N, 1), order=2)
        assert ei.value.status == P.PP_EINVAL
        with pytest.raises(P.PPError) as ei:
            h.window_solve(0.5, sys.N + 1)
        assert ei.value.status == P.PP_EINVAL
    with P.Handle.from_system(sys, order=2, max_cycles=1) as h:
        e, vec, f, info = h.window_solve(0.5, 6, allow_unconverged=True)
        assert info["status"] == P.PP_ENOTCONV
        assert np.all(np.isfinite(e))


def test_window_batch_matches_single_and_oracle(P):
    """Windows solved together (shared product passes) agree with the oracle and with solo solves."""
    sys = gen(7, 12, 40, 100)
    omegas = [0.45, 0.8, 1.1, 1.6]
    with P.Handle.from_system(sys, order=2) as h:
        eb, vb, fb, infos = h.window_solve_batch(omegas, 6)
        solo = [h.window_solve(w, 6) for w in omegas]
    for k, w in enumerate(omegas):
        _check_window(sys, 2, w, 6, eb[k], vb[k], fb[k], infos[k])
        np.testing.assert_allclose(eb[k], solo[k][0], rtol=0, atol=1e-10)
    with P.Handle.from_system(sys, order=2) as h:
        eb2, _, fb2, _ = h.window_solve_batch(omegas, 6)
    assert np.array_equal(eb, eb2) and np.array_equal(fb, fb2)


def test_fp32_products_within_single_precision(P):
    """FP32 contractions + FP64 diagonal/assembly: products agree with the oracle to FP32 accuracy."""
    torch = pytest.importorskip("torch")
    sys = _sys("mid")
    X = random_block(5, sys.N, 2)
    V = torch.tensor(np.concatenate([X[:, 0], X[:, 1]]), dtype=torch.float64, device="cuda")
    k = V.shape[0]
    outs = [torch.empty_like(V) for _ in range(6)]
    A, B, S = dense.assemble(sys, 2)
    with P.Handle.from_system(sys, order=2, precision=P.PP_FP32) as h:
        h.products(V, outs[0], outs[1], outs[2], fp32=False)
        h.products(V, outs[3], outs[4], outs[5], fp32=True)
    Vh = V.cpu().numpy()
    ref = [(A @ Vh.T).T, (B @ Vh.T).T, (S @ Vh.T).T]
    for j in range(3):
        np.testing.assert_allclose(outs[j].cpu().numpy(), ref[j], rtol=0, atol=1e-12 * np.abs(ref[j]).max())
        corr = ref[j] - (Vh * np.diag(A if j == 0 else (B if j == 1 else S))) if j < 2 else ref[j] - Vh
        err = np.abs(outs[3 + j].cpu().numpy() - ref[j]).max()
        assert err <= 2e-6 * np.abs(corr).max() + 1e-14, (j, err, np.abs(corr).max())


@pytest.mark.parametrize("name", ["mid", "ragged", "pad"])
@pytest.mark.parametrize("store", [1, 0])
def test_split_bf16_products(P, name, store):
    """Split-BF16 amplitude contraction (FP32 elsewhere, FP64 diagonal and assembly): the
    products agree with the oracle to the split's accuracy, a relative 2^-16 per product,
    on the parts beyond the diagonal; amplitudes stored or rebuilt in strips (then their
    integrals are split-BF16 products too), on a system whose particle-hole dimension and
    auxiliary size are whole 8-value chunks, on one where neither is, and on one whose
    rows are padded past a 4 KiB multiple."""
    torch = pytest.importorskip("torch")
    sys = _sys(name)
    print(f"[sbf16 products] system={name} store={store} N={sys.N} naux={sys.naux}", flush=True)
    X = random_block(5, sys.N, 2)
    V = torch.tensor(np.concatenate([X[:, 0], X[:, 1]]), dtype=torch.float64, device="cuda")
    outs = [torch.empty_like(V) for _ in range(3)]
    A, B, S = dense.assemble(sys, 2)
    A1, B1, _ = dense.assemble(sys, 1)
    with P.Handle.from_system(sys, order=2, precision=P.PP_SPLIT_BF16, store_amplitudes=store,
                              strip_rows=3) as h:
        h.products(V, outs[0], outs[1], outs[2], fp32=True)
    Vh = V.cpu().numpy()
    ref = [(A @ Vh.T).T, (B @ Vh.T).T, (S @ Vh.T).T]
    second = [((A - A1) @ Vh.T).T, ((B - B1) @ Vh.T).T, ref[2] - Vh]
    for j in range(3):
        err = np.abs(outs[j].cpu().numpy() - ref[j]).max()
        assert err <= 1e-4 * np.abs(second[j]).max() + 1e-12, (j, err, np.abs(second[j]).max())


@pytest.mark.parametrize("prec", ["fp32", "sbf16"])
@pytest.mark.parametrize("omega0,nr", [(0.45, 8), (1.1, 8)])
def test_window_mixed_precision(P, omega0, nr, prec):
    """FP32 (or split-BF16 amplitude) subspace products with FP64 restarts and FP64 residual
    acceptance meet the FP64 bar."""
    sys = gen(7, 12, 40, 100)
    with P.Handle.from_system(sys, order=2, precision=P.PP_FP32 if prec == "fp32" else P.PP_SPLIT_BF16) as h:
        e, vec, f, info = h.window_solve(omega0, nr)
    _check_window(sys, 2, omega0, nr, e, vec, f, info)
    assert np.all(info["residual"] <= 1e-9)


@pytest.mark.parametrize("prec", ["fp64", "sbf16"])
def test_window_passes_capped(P, prec):
    """Product passes capped at 7 vectors (pass_vectors), amplitudes rebuilt in strips of
    5 occupied rows: each window's 20-vector requests run as passes of equal size, every
    pass rebuilding the strips; two batched windows still match the oracle."""
    sys = gen(7, 12, 40, 100)
    pp = {"fp64": P.PP_FP64, "sbf16": P.PP_SPLIT_BF16}[prec]
    print(f"[window] passes capped at 7 vectors, {prec}", flush=True)
    with P.Handle.from_system(sys, order=2, store_amplitudes=0, strip_rows=5, pass_vectors=7, precision=pp) as h:
        e, vec, f, infos = h.window_solve_batch([0.45, 1.1], 8)
    for w, (omega0, nr) in enumerate(((0.45, 8), (1.1, 8))):
        _check_window(sys, 2, omega0, nr, e[w], vec[w], f[w], infos[w])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "sbf16"])
def test_window_survey_completeness(P, precision):
    """The full 40/160/600 workload in the launch configuration the benchmark times
    (amplitudes stored, windows batched): 24 windows across the spectrum, each must
    return exactly the oracle's 10 roots nearest omega0 (no root missed, none
    substituted), to 1e-8 Ha.  Mixed precision runs every third window."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mp2_o40_v160_x600.json")))
    survey = g["survey"] if precision == "fp64" else g["survey"][::3]
    from synth.gen import gen_config
    sys = gen_config("mp2_o40_v160_x600")
    prec = {"fp64": P.PP_FP64, "fp32": P.PP_FP32, "sbf16": P.PP_SPLIT_BF16}[precision]
    print(f"[survey] {len(survey)} windows, {precision}", flush=True)
    with P.Handle.from_system(sys, order=2, store_amplitudes=1, precision=prec) as h:
        for b0 in range(0, len(survey), 8):
            part = survey[b0:b0 + 8]
            e, _, _, infos = h.window_solve_batch([w["omega0"] for w in part], 10, vectors=False, osc=False)
            for k, w in enumerate(part):
                np.testing.assert_allclose(e[k], w["energies"], rtol=0, atol=1e-8,
                                           err_msg=f"window {w['omega0']:.4f}")
                assert np.all(infos[k]["converged"] == 1)
            print(f"[survey] windows {b0}..{b0 + len(part) - 1} ok", flush=True)


def test_window_tda(P):
    """Tamm-Dancoff windows (B = 0, A x = omega S x) at second order against the oracle."""
    sys = gen(7, 12, 40, 100)
    A, B, S = dense.assemble(sys, 2)
    for omega0, nr in ((0.45, 6), (1.1, 6)):
        with P.Handle.from_system(sys, order=2, tda=1) as h:
            e, vec, f, info = h.window_solve(omega0, nr)
        e_ref, X_ref, Y_ref, f_ref = pencil.window_solve(A, 0.0 * B, S, sys.dip, omega0, nr)
        np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-8)
        big = f_ref >= 1e-4 * f_ref.max()
        np.testing.assert_allclose(f[big], f_ref[big], rtol=1e-5)
        assert np.abs(vec[:, 1]).max() < 1e-10  # Y = 0
        assert np.all(info["converged"] == 1)


def test_window_order0_exact(P):
    """Zeroth order: roots are the orbital-energy differences, f = (4/3) D sum_x mu_x^2."""
    sys = gen(5, 6, 22, 40)
    D = (sys.eps_v[None, :] - sys.eps_o[:, None]).ravel()
    mu2 = np.sum(sys.dip.reshape(3, -1) ** 2, axis=0)
    with P.Handle.from_system(sys, order=0) as h:
        e, vec, f, info = h.window_solve(1.0, 6)
    idx = np.argsort(np.abs(D - 1.0), kind="stable")[:6]
    idx = idx[np.argsort(D[idx])]
    np.testing.assert_allclose(e, D[idx], rtol=0, atol=1e-12)
    np.testing.assert_allclose(f, (4.0 / 3.0) * D[idx] * mu2[idx], rtol=1e-10, atol=1e-14)


def test_window_correlated_property_vector(P):
    """Oscillator strengths from the correlated property vector F = S mu (second order)
    against the oracle; below second order S = 1 and they equal the plain ones."""
    sys = gen(7, 12, 40, 100)
    A, B, S = dense.assemble(sys, 2)
    with P.Handle.from_system(sys, order=2, correlated_f=1) as h:
        e, vec, f, info = h.window_solve(1.1, 8)
    e_ref, X_ref, Y_ref, f_ref = pencil.window_solve(A, B, S, sys.dip, 1.1, 8, correlated_f=True)
    _, _, _, f_plain = pencil.window_solve(A, B, S, sys.dip, 1.1, 8)
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-8)
    big = f_ref >= 1e-4 * f_ref.max()
    np.testing.assert_allclose(f[big], f_ref[big], rtol=1e-5)
    assert np.abs(f_ref - f_plain).max() > 1e-6 * f_ref.max()  # the correction is visible
    sys1 = gen(1, 8, 24, 64)
    with P.Handle.from_system(sys1, order=1, correlated_f=1) as h:
        e1, _, f1, _ = h.window_solve(0.5, 6)
    with P.Handle.from_system(sys1, order=1) as h:
        e0, _, f0, _ = h.window_solve(0.5, 6)
    np.testing.assert_allclose(f1, f0, rtol=1e-12)


def test_exciton_dos_matches_oracle(P):
    """Counts per bin bit-exact (same half-open rule, same FP64 difference), squared-dipole
    sums to rounding; bins that cut through the spectrum and empty bins included."""
    sys = gen(7, 12, 40, 100)
    dE = (sys.eps_v[None, :] - sys.eps_o[:, None]).ravel()
    edges = np.concatenate([[dE.min() - 0.5], np.linspace(dE.min(), dE.max(), 37), [dE.max() + 1e-12, 9.0]])
    edges = np.unique(edges)
    with P.Handle.from_system(sys, order=1) as h:
        counts, mu2 = h.exciton_dos(edges)
    c_ref, m_ref = pencil.exciton_dos(sys.eps_o, sys.eps_v, sys.dip, edges)
    np.testing.assert_array_equal(counts, c_ref)
    np.testing.assert_allclose(mu2, m_ref, rtol=1e-12, atol=1e-15)


def test_spectrum_broadening(P):
    """pp_spectrum (on the device): each root contributes a unit-area Lorentzian times its
    oscillator strength; the integral over a wide grid is the sum of strengths and an
    isolated peak has height f/(pi eta)."""
    e = np.array([0.5, 0.9, 0.905, 2.0])
    f = np.array([0.1, 0.02, 0.3, 0.05])
    eta = 2e-3
    w = np.linspace(-50.0, 60.0, 2_000_001)
    s = P.spectrum(e, f, w, eta)
    integral = np.sum(0.5 * (s[1:] + s[:-1]) * np.diff(w))
    tails = (f.sum() * 2 * eta / np.pi) * (1 / 50.0)  # the Lorentzian mass outside the grid, to first order
    assert abs(integral - f.sum()) < tails
    peak = P.spectrum(e, f, np.array([2.0]), eta)[0]
    assert abs(peak - f[3] / (np.pi * eta)) < 1e-3 * peak


@pytest.mark.parametrize("order", [1, 2])
def test_response_from_windows_matches_resolvent(P, order):
    """The propagator Pi(omega + i eta) of the library (pp_response), assembled from the
    roots of window solves that together cover the whole spectrum of the 8/24/64 system
    (192 roots; windows of 16 roots at every 8th oracle root and the last, the union
    deduplicated),
    against the oracle's resolvent form F^T (w Sigma - M)^-1 F by dense complex solves on
    a frequency grid, real and imaginary parts, to 1e-8 of the largest value; the union of
    the windows is exactly the oracle's set of roots."""
    sys_ = gen(1, 8, 24, 64)
    A, B, S = dense.assemble(sys_, order)
    w_all, _, _ = pencil.solve_all(A, B, S)
    centers = list(w_all[0::8]) + [w_all[-1]]
    got_e, got_f = [], []
    with P.Handle.from_system(sys_, order=order) as h:
        E, _, F, infos = h.window_solve_batch(centers, 16, vectors=False, osc=True)
    for k in range(len(centers)):
        assert np.all(infos[k]["converged"] == 1)
        got_e.extend(E[k])
        got_f.extend(F[k])
    got_e, got_f = np.array(got_e), np.array(got_f)
    order_ = np.argsort(got_e, kind="stable")
    got_e, got_f = got_e[order_], got_f[order_]
    keep = np.concatenate([[True], np.diff(got_e) > 1e-9])
    got_e, got_f = got_e[keep], got_f[keep]
    assert len(got_e) == len(w_all) == sys_.N
    np.testing.assert_allclose(got_e, w_all, rtol=0, atol=1e-8)
    grid = np.linspace(0.0, 3.5, 351)
    for eta in (0.01, 0.05):
        pi_lib = P.response(got_e, got_f, grid, eta)
        pi_ref = pencil.response_resolvent(A, B, S, sys_.dip, grid, eta)
        scale = np.abs(pi_ref).max()
        np.testing.assert_allclose(pi_lib.real, pi_ref.real, rtol=0, atol=1e-8 * scale)
        np.testing.assert_allclose(pi_lib.imag, pi_ref.imag, rtol=0, atol=1e-8 * scale)
    # static limit (eta = 0, omega = 0): minus the static polarizability
    p0 = P.response(got_e, got_f, np.array([0.0]), 0.0)[0]
    ref0 = pencil.response_resolvent(A, B, S, sys_.dip, [0.0], 0.0)[0]
    assert abs(p0.real - ref0.real) < 1e-8 * abs(ref0.real) and p0.imag == 0.0
