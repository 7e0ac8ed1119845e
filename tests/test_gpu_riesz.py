"""Riesz-projector window isolation on the GPU, through the C ABI, against the oracle.

* The contour filter (trapezoidal quadrature of (z Sigma - M)^-1 Sigma, shifted systems
  solved by preconditioned COCG on the device) against the oracle's dense quadrature
  with exact solves, on random blocks: to 1e-8 of the largest element with solves to
  1e-12 (the solve error is amplified by at most the condition number of the shifted
  systems, about radius / distance of the nearest node to a root).
* On exact eigenvectors of the pencil the device filter reproduces the closed form
  1 / (1 + x^(2n)) of the rule.
* Window solves with method = PP_RIESZ return the oracle's window (plain definition):
  energies to 1e-8 Ha, strengths to 1e-5 relative, S-normalised vectors up to sign.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import gen
from synth.gen import random_block
from oracle import dense, pencil, riesz

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2512_09811_amd as P
    P.lib()
    return P


def _blocks(V):
    """[2N][m] columns -> torch device [m][2][N]."""
    N = V.shape[0] // 2
    return torch.tensor(np.ascontiguousarray(V.T.reshape(-1, 2, N)), device="cuda")


@pytest.mark.parametrize("order,nodes", [(1, 4), (2, 6), (2, 8)])
def test_contour_filter_matches_dense_quadrature(P, order, nodes):
    sys = gen(13, 6, 20, 48)
    print(f"[riesz filter] order={order} nodes={nodes} o={sys.o} v={sys.v}", flush=True)
    A, B, S = dense.assemble(sys, order)
    M, Sig = riesz.pencil_matrices(A, B, S)
    omega, _, _ = pencil.solve_all(A, B, S)
    c = float(np.median(omega))
    r = 0.1 * float(omega[-1] - omega[0])
    V = random_block(3, sys.N, 3).reshape(3, 2 * sys.N).T          # [2N][3]
    ref = riesz.riesz_apply(M, Sig, V, c, r, nodes)
    with P.Handle.from_system(sys, order=order) as h:
        dV = _blocks(V)
        out = torch.empty_like(dV)
        it, worst = h.riesz_filter(dV, out, c, r, nodes, tol=1e-12, maxit=400)
    got = out.cpu().numpy().reshape(3, 2 * sys.N).T
    assert worst <= 1e-12 and it < 400
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-8 * np.abs(ref).max())


def test_contour_filter_on_eigenvectors_is_rational_filter(P):
    sys = gen(17, 5, 18, 40)
    A, B, S = dense.assemble(sys, 2)
    omega, X, Y = pencil.solve_all(A, B, S)
    c = float(omega[len(omega) // 3])
    r = 0.08 * float(omega[-1] - omega[0])
    pick = np.argsort(np.abs(omega - c))[[0, 1, 5, 12, 45]]
    Z = np.vstack([X[:, pick], Y[:, pick]])
    n = 6
    with P.Handle.from_system(sys, order=2) as h:
        dZ = _blocks(Z)
        out = torch.empty_like(dZ)
        h.riesz_filter(dZ, out, c, r, n, tol=1e-12, maxit=400)
    got = out.cpu().numpy().reshape(len(pick), 2 * sys.N).T
    rho = riesz.filter_value((omega[pick] - c) / r, n)
    assert rho.max() > 0.9 and rho.min() < 1e-3
    np.testing.assert_allclose(got, Z * rho, rtol=0, atol=1e-9 * np.abs(Z).max())


def _check(sys, order, omega0, nr, e, vec, f, info):
    A, B, S = dense.assemble(sys, order)
    e_ref, X_ref, Y_ref, f_ref = pencil.window_solve(A, B, S, sys.dip, omega0, nr)
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-8)
    big = f_ref >= 1e-4 * f_ref.max()
    np.testing.assert_allclose(f[big], f_ref[big], rtol=1e-5)
    np.testing.assert_allclose(f[~big], f_ref[~big], rtol=0, atol=1e-9)
    for q in range(nr):
        ov = vec[q, 0] @ S @ X_ref[:, q] - vec[q, 1] @ S @ Y_ref[:, q]
        assert abs(abs(ov) - 1.0) < 1e-6, (q, ov)
    assert np.all(info["converged"] == 1)


@pytest.mark.parametrize("order,omega0,nr", [(1, 0.5, 6), (2, 0.8, 8), (2, 1.3, 5)])
def test_window_riesz_matches_oracle(P, order, omega0, nr):
    sys = gen(7, 12, 40, 100, b_scale=0.3)
    print(f"[riesz window] order={order} omega0={omega0} nr={nr}", flush=True)
    with P.Handle.from_system(sys, order=order, method=P.PP_RIESZ) as h:
        e, vec, f, info = h.window_solve(omega0, nr)
    _check(sys, order, omega0, nr, e, vec, f, info)


def test_window_riesz_batch_and_mixed_precision(P):
    """Several windows in one call share product passes; FP32 products for the filter
    with the FP64 refinement still give the oracle's windows."""
    sys = gen(1, 8, 24, 64)
    oms = [0.45, 0.9]
    for prec in (P.PP_FP64, P.PP_FP32):
        print(f"[riesz batch] precision={prec}", flush=True)
        with P.Handle.from_system(sys, order=2, method=P.PP_RIESZ, precision=prec) as h:
            E, V, F, infos = h.window_solve_batch(oms, 6)
        for w, om in enumerate(oms):
            _check(sys, 2, om, 6, E[w], V[w], F[w], infos[w])


def test_window_riesz_survey(P):
    """Seven windows from 0.4 to 1.6 Ha (6 roots each) on three 16/64/192 second-order
    systems, Riesz mode, batched: every window equals the oracle's."""
    bad = []
    for seed in (1, 2, 3):
        s = gen(seed, 16, 64, 192)
        A, B, S = dense.assemble(s, 2)
        om, _, _ = pencil.solve_all(A, B, S)
        oms = np.linspace(0.4, 1.6, 7)
        print(f"[riesz survey] seed {seed}", flush=True)
        with P.Handle.from_system(s, order=2, method=P.PP_RIESZ) as h:
            E, _, _, infos = h.window_solve_batch(oms, 6, vectors=False, osc=False, allow_unconverged=True)
        for w, w0 in enumerate(oms):
            ref = om[pencil.select_window(om, w0, 6)]
            if not (np.abs(E[w] - ref).max() < 1e-8 and np.all(infos[w]["converged"] == 1)):
                bad.append((seed, float(w0)))
    assert not bad, bad
