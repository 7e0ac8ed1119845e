"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them re-types an oracle formula: they
compare against an independent route (brute-force Fock space, spin-orbital
algebra, a textbook special case, a closed form or an identity).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from synth import gen
from oracle import dense, fockspace, folded, pencil, spinorb


# ---------------------------------------------------------------------------
# P6: brute-force Fock space vs the spin-orbital closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("no,nv,seed", [(2, 3, 1), (3, 3, 2), (2, 4, 3), (2, 2, 4)])
def test_p6_spinorbital_forms_equal_defining_expectation_values(no, nv, seed):
    """S2, A2 (symmetrized, W-cross terms included), B2 and first order vs brute force."""
    eps, _, V = spinorb.spinless_system(seed, no, nv)
    r = fockspace.MP2Response(eps, no, V)
    S0, S2 = r.metric()
    A0, A1, A2 = r.a_block()
    B0, B1, B2 = r.b_block()
    Ac = [spinorb.assemble(eps, no, V, k) for k in (0, 1, 2)]
    scale = max(np.abs(A2).max(), np.abs(B2).max(), np.abs(S2).max())
    assert scale > 1e-5                     # the second-order pieces are not trivially zero
    np.testing.assert_allclose(S0, Ac[0][2], atol=1e-14)
    np.testing.assert_allclose(A0, Ac[0][0], atol=1e-14)
    np.testing.assert_allclose(A0 + A1, Ac[1][0], atol=1e-14)
    np.testing.assert_allclose(B1, Ac[1][1], atol=1e-14)
    np.testing.assert_allclose(B0, 0, atol=1e-15)
    np.testing.assert_allclose(S2, Ac[2][2] - Ac[1][2], atol=1e-14)
    np.testing.assert_allclose(A2, Ac[2][0] - Ac[1][0], atol=1e-14)
    np.testing.assert_allclose(B2, Ac[2][1] - Ac[1][1], atol=1e-14)


def test_p6_first_order_is_tdhf_and_fock_is_diagonal():
    """First order equals textbook TDHF: A1 = <aj||ib>, B1 = <ab||ij>; Brillouin holds."""
    eps, no, V = spinorb.spinless_system(11, 2, 3)
    r = fockspace.MP2Response(eps, no, V)
    assert r.brillouin_max() < 1e-14
    _, A1, _ = r.a_block()
    _, B1, _ = r.b_block()
    nv = len(eps) - no
    for i in range(no):
        for a in range(nv):
            for j in range(no):
                for b in range(nv):
                    assert abs(A1[i * nv + a, j * nv + b] - V[no + a, j, i, no + b]) < 1e-14
                    assert abs(B1[i * nv + a, j * nv + b] - V[no + a, no + b, i, j]) < 1e-14


def test_p6_literal_reading_differs_from_r2():
    """The H0-only (literal) second-order A is 1/2(Delta_ai + Delta_bj) S2; the W-cross part is not zero."""
    eps, no, V = spinorb.spinless_system(5, 2, 3)
    r = fockspace.MP2Response(eps, no, V)
    h0_part, w_part = r.a2_parts()
    _, S2 = r.metric()
    nv = len(eps) - no
    delta = (eps[no:][None, :] - eps[:no][:, None]).reshape(-1)
    np.testing.assert_allclose(h0_part, 0.5 * (delta[:, None] + delta[None, :]) * S2, atol=1e-14)
    assert np.abs(w_part).max() > 1e-4


@pytest.mark.parametrize("no,nv,seed", [(2, 3, 1), (3, 2, 4)])
def test_p10_mp2_energy_brute_force(no, nv, seed):
    """<0|W_N R0 W_N|0> from explicit matrices equals 1/4 sum t <ij||ab> (textbook MP2)."""
    eps, _, V = spinorb.spinless_system(seed, no, nv)
    r = fockspace.MP2Response(eps, no, V)
    assert abs(r.mp2_energy() - spinorb.mp2_energy(eps, no, V)) < 1e-15
    # Psi1 has only doubly excited components
    for k, d in enumerate(r.fs.dets):
        holes = bin(((1 << no) - 1) & ~d).count("1")
        if abs(r.psi1[k]) > 1e-14:
            assert holes == 2


# ---------------------------------------------------------------------------
# P7: spin adaptation (spatial closed-shell singlet vs spin orbitals)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("o,v,naux,seed", [(2, 3, 5, 1), (3, 4, 7, 2), (1, 2, 3, 3)])
def test_p7_singlet_projection_equals_spin_adapted(o, v, naux, seed):
    sys = gen(seed, o, v, naux, b_scale=0.6)
    eps_so, no_so, V = spinorb.spinorbital_system(sys)
    for order in (1, 2):
        Aso, Bso, Sso = spinorb.assemble(eps_so, no_so, V, order)
        A, B, S = dense.assemble(sys, order)
        for Mso, M in ((Aso, A), (Bso, B), (Sso, S)):
            sing, _ = spinorb.singlet_triplet_projection(Mso, o, v)
            np.testing.assert_allclose(sing, M, atol=1e-14)
    assert abs(dense.mp2_energy(sys) - spinorb.mp2_energy(eps_so, no_so, V)) < 1e-14


def test_p7_brute_force_closed_shell_singlet():
    """Closed-shell system through the Fock-space route directly, singlet-projected."""
    o, v = 2, 3
    sys = gen(9, o, v, 4, b_scale=0.6)
    eps_so, no_so, V = spinorb.spinorbital_system(sys)
    r = fockspace.MP2Response(eps_so, no_so, V)
    S0, S2 = r.metric()
    A0, A1, A2 = r.a_block()
    _, B1, B2 = r.b_block()
    A, B, S = dense.assemble(sys, 2)
    np.testing.assert_allclose(spinorb.singlet_triplet_projection(A0 + A1 + A2, o, v)[0], A, atol=1e-14)
    np.testing.assert_allclose(spinorb.singlet_triplet_projection(B1 + B2, o, v)[0], B, atol=1e-14)
    np.testing.assert_allclose(spinorb.singlet_triplet_projection(S0 + S2, o, v)[0], S, atol=1e-14)


def test_p4_two_level_closed_form_against_brute_force():
    """o = v = 1: omega = sqrt(A^2 - B^2)/S with the scalar second-order A, B, S.

    The scalars are the singlet projection of the brute-force Fock-space
    matrices (4 spin orbitals, 2 electrons); the pencil solver must return the
    closed-form root.
    """
    sys = gen(21, 1, 1, 3, b_scale=0.8)
    eps_so, no_so, V = spinorb.spinorbital_system(sys)
    r = fockspace.MP2Response(eps_so, no_so, V)
    S0, S2 = r.metric()
    A0, A1, A2 = r.a_block()
    _, B1, B2 = r.b_block()
    a = spinorb.singlet_triplet_projection(A0 + A1 + A2, 1, 1)[0][0, 0]
    b = spinorb.singlet_triplet_projection(B1 + B2, 1, 1)[0][0, 0]
    s = spinorb.singlet_triplet_projection(S0 + S2, 1, 1)[0][0, 0]
    w_closed = np.sqrt(a * a - b * b) / s
    A, B, S = dense.assemble(sys, 2)
    w, X, Y = pencil.solve_all(A, B, S)
    assert abs(w[0] - w_closed) < 1e-14
    # first order: omega = sqrt((A - B)(A + B))
    a1 = spinorb.singlet_triplet_projection(A0 + A1, 1, 1)[0][0, 0]
    b1 = spinorb.singlet_triplet_projection(B1, 1, 1)[0][0, 0]
    w1, _, _ = pencil.solve_all(*dense.assemble(sys, 1))
    assert abs(w1[0] - np.sqrt((a1 - b1) * (a1 + b1))) < 1e-14


# ---------------------------------------------------------------------------
# P1, P2, P3, P5: special cases and structure
# ---------------------------------------------------------------------------
def test_p1_zero_integrals_give_orbital_energy_differences():
    sys = gen(1, 8, 24, 64).scaled(0.0)
    for order in (0, 1, 2):
        A, B, S = dense.assemble(sys, order)
        w, X, Y = pencil.solve_all(A, B, S)
        delta = np.sort((sys.eps_v[None, :] - sys.eps_o[:, None]).reshape(-1))
        assert np.array_equal(w, np.sqrt(delta * delta)) or np.abs(w - delta).max() < 1e-15
        e, Xw, Yw, f = pencil.window_solve(A, B, S, sys.dip, 0.5, 6)
        d = (sys.eps_v[None, :] - sys.eps_o[:, None]).reshape(-1)
        pick = np.sort(np.argsort(np.abs(d - 0.5), kind="stable")[:6])
        pick = pick[np.argsort(d[pick])]
        np.testing.assert_allclose(e, d[pick], rtol=0, atol=1e-15)
        mu2 = np.sum(sys.dip.reshape(3, -1) ** 2, axis=0)
        np.testing.assert_allclose(f, (4.0 / 3.0) * d[pick] * mu2[pick], rtol=1e-13)


def test_p2_symmetry_and_first_order_metric():
    sys = gen(1, 8, 24, 64)
    for order in (1, 2):
        A, B, S = dense.assemble(sys, order)
        for M in (A, B, S):
            assert np.abs(M - M.T).max() <= 1e-14 * np.abs(M).max()
        if order == 1:
            assert np.array_equal(S, np.eye(len(S)))
        assert np.linalg.eigvalsh(S).min() > 0
        assert np.linalg.eigvalsh(A - B).min() > 0 and np.linalg.eigvalsh(A + B).min() > 0


def test_p3_plus_minus_pairs_general_eig():
    sys = gen(1, 8, 24, 64)
    for order in (1, 2):
        M, Sig = dense.build_M(sys, order)
        w, imax = pencil.pencil_eigvals_general(M, Sig)
        assert imax < 1e-12
        np.testing.assert_allclose(np.sort(w), np.sort(-w), atol=1e-12)
        om, _, _ = pencil.solve_all(*dense.assemble(sys, order))
        np.testing.assert_allclose(np.sort(np.concatenate([om, -om])), w, atol=1e-12)


def test_p5_tda_limit_is_generalized_symmetric_eig():
    sys = gen(3, 6, 20, 40, b_scale=0.3)
    A, B, S = dense.assemble(sys, 2)
    w, _, _ = pencil.solve_all(A, np.zeros_like(B), S)
    np.testing.assert_allclose(w, sla.eigh(A, S, eigvals_only=True), rtol=1e-13)


def test_p11_particle_conservation():
    sys = gen(4, 6, 18, 30, b_scale=0.5)
    it = dense.second_order_intermediates(sys)
    assert abs(np.trace(it["Go"]) - np.trace(it["Gv"])) < 1e-14 * max(1.0, np.trace(it["Gv"]))
    assert np.trace(it["Gv"]) > 0


def test_p12_perturbative_limit():
    """omega(lam) = Delta + lam A1_diag + O(lam^2) for non-degenerate Delta (integrals scaled by lam)."""
    sys = gen(6, 3, 5, 8)
    A1, _, _ = dense.assemble(sys.scaled(1.0), 1)
    d = (sys.eps_v[None, :] - sys.eps_o[:, None]).reshape(-1)
    order = np.argsort(d)
    a1 = np.diag(A1)[order] - d[order]
    for lam in (1e-3, 1e-4):
        w, _, _ = pencil.solve_all(*dense.assemble(sys.scaled(np.sqrt(lam)), 2))
        slope = (w - d[order]) / lam
        np.testing.assert_allclose(slope, a1, rtol=0, atol=50 * lam * np.abs(a1).max() + 1e-9)


# ---------------------------------------------------------------------------
# Strengths, solver, variance
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [1, 2])
def test_strength_sum_rule(order):
    """sum_n omega_n (mu.(X+Y)_n)^2 = mu^T S^-1 (A - B) S^-1 mu (completeness of the pencil)."""
    sys = gen(8, 6, 20, 40, b_scale=0.4)
    A, B, S = dense.assemble(sys, order)
    w, X, Y = pencil.solve_all(A, B, S)
    f = pencil.oscillator_strengths(w, X, Y, sys.dip)
    Si = np.linalg.inv(S)
    mu = sys.dip.reshape(3, -1)
    rhs = (4.0 / 3.0) * sum(m @ Si @ (A - B) @ Si @ m for m in mu)
    assert abs(f.sum() - rhs) < 1e-12 * rhs
    # the S-normalization every root carries
    np.testing.assert_allclose(np.einsum("ik,ij,jk->k", X, S, X) - np.einsum("ik,ij,jk->k", Y, S, Y), 1.0,
                               atol=1e-12)


def test_alpha_weight_minimizes_folded_quotient():
    rng = np.random.default_rng(0)
    for _ in range(50):
        Z = rng.standard_normal((12, 12))
        Z = Z + Z.T
        v = rng.standard_normal(12)
        v /= np.linalg.norm(v)
        d = rng.standard_normal(12)

        def rho(a):
            x = v + a * d
            return (x @ Z @ Z @ x) / (x @ x)

        y, zd = Z @ v, Z @ d
        al = folded.alpha_weight(y @ y, 2 * y @ zd, zd @ zd, 2 * v @ d, d @ d)
        grid = np.linspace(-20, 20, 40001)
        best = min(rho(a) for a in grid)
        assert rho(al) <= best + 1e-9


@pytest.mark.parametrize("order,o,v,naux,seed,omega0,nr", [
    (1, 8, 24, 64, 1, 0.5, 6), (2, 8, 24, 64, 1, 0.5, 6), (2, 12, 40, 100, 7, 0.7, 8), (2, 12, 40, 100, 7, 1.3, 8)])
def test_p8_folded_roots_equal_full_diagonalization(order, o, v, naux, seed, omega0, nr):
    sys = gen(seed, o, v, naux)
    A, B, S = dense.assemble(sys, order)
    e, X, Y, f = pencil.window_solve(A, B, S, sys.dip, omega0, nr)
    th, Xf, Yf, info = folded.folded_window_solve(A, B, S, omega0, nr)
    assert info["converged"]
    np.testing.assert_allclose(th, e, rtol=0, atol=1e-10)
    f2 = pencil.oscillator_strengths(th, Xf, Yf, sys.dip)
    np.testing.assert_allclose(f2, f, rtol=1e-6, atol=1e-12)


def test_p9_variance_vanishes_for_converged_vectors():
    """sigma^2 = rho_{A^2} - rho_A^2 -> 0 and sqrt(rho_{A^2}) vs rho_A has unit slope on eigenvectors."""
    sys = gen(1, 8, 24, 64)
    A, B, S = dense.assemble(sys, 1)
    lam, U = np.linalg.eigh(A)
    var = np.array([pencil.variance(A, U[:, k]) for k in range(len(lam))])
    assert var.max() < 1e-14
    rA = np.array([U[:, k] @ A @ U[:, k] for k in range(len(lam))])
    rA2 = np.array([np.sqrt(U[:, k] @ A @ A @ U[:, k]) for k in range(len(lam))])
    slope = np.polyfit(rA, rA2, 1)[0]
    assert abs(slope - 1.0) < 1e-10
    # a perturbed vector has a strictly positive variance
    x = U[:, 3] + 1e-2 * U[:, 7]
    assert pencil.variance(A, x) > 1e-8


def test_first_order_rows_match_dense_assembly():
    """The sampled-row oracle used at full sizes agrees with the dense first-order
    assembly (a second, independent route through the same definitions)."""
    from oracle import columns
    sys_ = gen(3, 5, 13, 29)
    A, B, S = dense.assemble(sys_, 1)
    rng = np.random.default_rng(0)
    V = rng.standard_normal((3, sys_.N))
    rows = [0, 7, 20, 64]
    Boo_i = [sys_.B_oo[:, r // sys_.v, :] for r in rows]
    Bvv_a = [sys_.B_vv[:, r % sys_.v, :] for r in rows]
    AV, BV = columns.first_order_rows(sys_.eps, sys_.o, sys_.v, sys_.B_ov, rows, Boo_i, Bvv_a, V)
    np.testing.assert_allclose(AV, (V @ A.T)[:, rows], rtol=0, atol=1e-14)
    np.testing.assert_allclose(BV, (V @ B.T)[:, rows], rtol=0, atol=1e-14)


def test_tda_pencil_matches_generalized_eigh():
    """Tamm-Dancoff (B = 0): the pencil route reduces to the generalized symmetric
    problem A x = omega S x (library routine scipy.linalg.eigh(A, S))."""
    sys_ = gen(4, 4, 9, 20, b_scale=0.4)
    A, B, S = dense.assemble(sys_, 2)
    w_ref, Xr = sla.eigh(A, S)
    for w0, nr in ((0.6, 4), (1.3, 5)):
        e, X, Y, f = pencil.window_solve(A, 0.0 * B, S, sys_.dip, w0, nr)
        idx = np.sort(np.argsort(np.abs(w_ref - w0), kind="stable")[:nr])
        np.testing.assert_allclose(e, w_ref[idx], rtol=0, atol=1e-12)
        assert np.abs(Y).max() < 1e-13
        np.testing.assert_allclose(np.einsum("nq,nm,mq->q", X, S, X), 1.0, atol=1e-12)


@pytest.mark.parametrize("no,nv,seed", [(2, 3, 1), (3, 3, 2), (2, 4, 3)])
def test_p6_property_vector_is_metric_times_dipole(no, nv, seed):
    """F_k = <[q_k, D]> over the MP2 ground state (brute force, D with oo, ov and vv
    blocks) equals S d_ov through second order: the oo and vv blocks of D drop out and
    the correlated property vector is the metric applied to the zeroth-order one."""
    eps, _, V = spinorb.spinless_system(seed, no, nv)
    r = fockspace.MP2Response(eps, no, V)
    n = no + nv
    Z = np.random.default_rng(seed + 50).standard_normal((n, n))
    d = 0.5 * (Z + Z.T)
    F0, F2 = r.property_vector(d)
    S0, S2 = r.metric()
    d_ov = np.array([d[i, no + a] for i in range(no) for a in range(nv)])
    assert np.abs(F2).max() > 1e-5
    np.testing.assert_allclose(F0, d_ov, atol=1e-14)
    np.testing.assert_allclose(F2, S2 @ d_ov, atol=1e-13)


def test_exciton_dos_invariants():
    """Every pair lands in exactly one bin of a covering grid; the squared-dipole sums add
    up to the total; a single pair fills exactly its own bin."""
    sys_ = gen(2, 6, 21, 30)
    dE = (sys_.eps_v[None, :] - sys_.eps_o[:, None]).ravel()
    edges = np.linspace(dE.min(), dE.max() + 1e-9, 13)
    counts, mu2 = pencil.exciton_dos(sys_.eps_o, sys_.eps_v, sys_.dip, edges)
    assert counts.sum() == sys_.N
    np.testing.assert_allclose(mu2.sum(), np.sum(sys_.dip ** 2), rtol=1e-13)
    one = gen(3, 1, 1, 4)
    d1 = one.eps_v[0] - one.eps_o[0]
    c1, m1 = pencil.exciton_dos(one.eps_o, one.eps_v, one.dip, np.array([d1 - 1, d1, d1 + 1]))
    np.testing.assert_array_equal(c1, [0, 1])
    np.testing.assert_allclose(m1, [0, np.sum(one.dip ** 2)], rtol=1e-14)


# ---------------------------------------------------------------------------
# Riesz projector (section connecting the method to the Riesz projector)
# ---------------------------------------------------------------------------
def _small_pencil(order=2, o=3, v=5, naux=12, seed=21):
    s = gen(seed, o, v, naux)
    A, B, S = dense.assemble(s, order)
    return s, A, B, S


@pytest.mark.parametrize("n", [2, 4, 8])
def test_riesz_trapezoid_filter_closed_form(n):
    """On every eigenvector of the pencil (both branches) the quadrature of the contour
    integral is the rational filter 1/(1 + x^(2n)) of x = (omega - c)/r: a closed form of
    the 2n-node rule, independent of how the shifted systems are solved."""
    from oracle import riesz
    _, A, B, S = _small_pencil()
    omega, X, Y = pencil.solve_all(A, B, S)
    M, Sig = riesz.pencil_matrices(A, B, S)
    c = float(omega[len(omega) // 2])
    r = 0.6 * float(omega[-1] - omega[0]) / 4
    Z = np.concatenate([np.vstack([X, Y]), np.vstack([Y, X])], axis=1)   # +omega and -omega
    w = np.concatenate([omega, -omega])
    PZ = riesz.riesz_apply(M, Sig, Z, c, r, n)
    rho = 1.0 / (1.0 + ((w - c) / r) ** (2 * n))
    assert rho.max() > 0.99 and rho.min() < 1e-3            # some roots inside, some far outside
    np.testing.assert_allclose(PZ, Z * rho, rtol=0, atol=1e-11 * np.abs(Z).max())


def test_riesz_projector_limit_is_spectral_projector():
    """With many nodes and a circle boundary in a spectral gap, the quadrature is the
    spectral projector: idempotent, with trace = number of enclosed roots."""
    from oracle import riesz
    _, A, B, S = _small_pencil(o=2, v=4, naux=10, seed=5)
    omega, _, _ = pencil.solve_all(A, B, S)
    M, Sig = riesz.pencil_matrices(A, B, S)
    gaps = np.diff(omega)
    g = int(np.argmax(gaps[: len(gaps) // 2 + 1]))
    c = float(omega[0]) - 1e-3
    r = 0.5 * (omega[g] + omega[g + 1]) - c
    P = riesz.riesz_apply(M, Sig, np.eye(M.shape[0]), c, r, 64)
    inside = int(np.sum(np.abs(omega - c) < r))
    assert inside == g + 1
    assert abs(np.trace(P) - inside) < 1e-8
    np.testing.assert_allclose(P @ P, P, atol=1e-8)


@pytest.mark.parametrize("order,omega0,nr", [(1, 0.5, 4), (2, 0.8, 6)])
def test_riesz_window_solve_equals_definition(order, omega0, nr):
    """Contour-filtered subspace iteration returns the window of the plain definition
    (all eigenpairs of the pencil, nearest roots): energies, S-normalised vectors."""
    from oracle import riesz
    s = gen(31, 6, 20, 48)
    A, B, S = dense.assemble(s, order)
    e_ref, X_ref, Y_ref, _ = pencil.window_solve(A, B, S, s.dip, omega0, nr)
    e, X, Y, it = riesz.riesz_window_solve(A, B, S, omega0, nr, nodes=8, tol=1e-11)
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-11)
    for k in range(nr):
        ov = X[:, k] @ S @ X_ref[:, k] - Y[:, k] @ S @ Y_ref[:, k]
        assert abs(abs(ov) - 1.0) < 1e-8, (k, ov)
    assert it < 60


@pytest.mark.parametrize("o,v,naux,seed,b_scale", [(5, 19, 23, 11, 0.5), (8, 24, 64, 1, 1.0)])
def test_second_order_rows_match_dense_assembly(o, v, naux, seed, b_scale):
    """Rows of the complete A, B, S through second order from the element form, one row
    at a time (oracle.columns.second_order_rows, the row oracle used where no dense matrix
    fits) equal the rows of the dense assembly (itself pinned against the brute-force Fock
    space, P6) for every row; the MP2 densities summed one occupied index at a time equal
    the dense ones; without the densities the B rows still come back complete."""
    from oracle import columns
    sys_ = gen(seed, o, v, naux, b_scale=b_scale)
    eps = np.concatenate([sys_.eps_o, sys_.eps_v])
    A, B, S = dense.assemble(sys_, 2)
    A1, B1, _ = dense.assemble(sys_, 1)
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((3, sys_.N))
    rows = list(range(sys_.N))
    dens = columns.mp2_densities(eps, o, v, sys_.B_ov)
    it = dense.second_order_intermediates(sys_)
    for key in ("Gv", "Ev", "Go", "Eo"):
        np.testing.assert_allclose(dens[key], it[key], rtol=0, atol=1e-14 * np.abs(it[key]).max())
    AV, BV, SV = columns.second_order_rows(eps, o, v, sys_.B_oo, sys_.B_ov, sys_.B_vv, rows, V, dens)
    for got, M, M1 in ((AV, A, A1), (BV, B, B1), (SV, S, np.eye(sys_.N))):
        ref = V @ M.T
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        second = V @ (M - M1).T
        assert np.abs(second).max() > 1e-6 * np.abs(ref).max()   # the second-order part is present
        np.testing.assert_allclose(got - V @ M1.T, second, rtol=0, atol=1e-11 * np.abs(second).max())
    _, BVb, _ = columns.second_order_rows(eps, o, v, sys_.B_oo, sys_.B_ov, sys_.B_vv, rows[:7], V)
    np.testing.assert_allclose(BVb, BV[:, :7], rtol=0, atol=1e-15 * np.abs(BV).max())


def test_b2_pp_ladder_factor_by_factor_equals_eri_form():
    """The two forms of the pp ladder in dense.b2_dense (through (ac|bd), and factor by
    factor for large n_vir) give the same B2."""
    sys_ = gen(3, 4, 14, 21, b_scale=0.7)
    tau = dense.second_order_intermediates(sys_)["tau"]
    a = dense.b2_dense(sys_, tau, ladder="eri")
    b = dense.b2_dense(sys_, tau, ladder="per_P")
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(a).max())
    assert np.abs(a).max() > 0


def test_select_window_ties_take_the_lower_root():
    """Window selection: the n roots nearest omega0; roots equidistant from omega0 (within
    the 1e-9 Ha resolution) go to the lower one; a root nearer by more than that wins."""
    om = np.array([0.2, 0.4, 0.45, 0.55, 0.6, 0.9])
    assert pencil.select_window(om, 0.5, 1).tolist() == [2]          # 0.45 and 0.55 tie -> 0.45
    assert pencil.select_window(om, 0.5, 2).tolist() == [2, 3]
    assert pencil.select_window(om, 0.5, 3).tolist() == [1, 2, 3]    # 0.4 and 0.6 tie -> 0.4
    assert pencil.select_window(om, 0.5, 4).tolist() == [1, 2, 3, 4]
    om2 = om.copy()
    om2[3] = 0.55 + 3e-10                                             # still a tie at 1e-9
    assert pencil.select_window(om2, 0.5, 1).tolist() == [2]
    om2[3] = 0.55 - 2e-9                                              # nearer by 2e-9 Ha
    assert pencil.select_window(om2, 0.5, 1).tolist() == [3]
    # result is ascending in omega whatever the input order
    perm = np.array([5, 3, 0, 4, 1, 2])
    assert sorted(om[perm][pencil.select_window(om[perm], 0.5, 3)].tolist()) == [0.4, 0.45, 0.55]


@pytest.mark.parametrize("order", [1, 2])
def test_response_resolvent_limits_and_poles(order):
    """The propagator from the resolvent of the pencil (one complex solve per frequency)
    against what fixes it independently of any eigen-decomposition: the static limit
    Pi(0) = -(4/3) sum_x mu_x^T (A + B)^-1 mu_x, the high-frequency limit
    w^2 Pi(w) -> (4/3) sum_x mu_x^T S^-1 (A - B) S^-1 mu_x (the strength sum rule), and the
    pole residues -eta Im Pi(w_k + i eta) -> f_k / (2 w_k) at an isolated root; then the
    spectral form over all roots equals it on a grid."""
    sys_ = gen(8, 6, 20, 40, b_scale=0.4)
    A, B, S = dense.assemble(sys_, order)
    mu = sys_.dip.reshape(3, -1)
    static = -(4.0 / 3.0) * sum(m @ np.linalg.solve(A + B, m) for m in mu)
    p0 = pencil.response_resolvent(A, B, S, sys_.dip, [0.0], 0.0)[0]
    assert abs(p0.imag) < 1e-14 and abs(p0.real - static) < 1e-11 * abs(static)
    Si = np.linalg.inv(S)
    trk = (4.0 / 3.0) * sum(m @ Si @ (A - B) @ Si @ m for m in mu)
    big = 1e4
    pinf = pencil.response_resolvent(A, B, S, sys_.dip, [big], 0.0)[0]
    assert abs(big * big * pinf.real - trk) < 1e-6 * trk
    w, X, Y = pencil.solve_all(A, B, S)
    f = pencil.oscillator_strengths(w, X, Y, sys_.dip)
    gaps = np.minimum(np.diff(w, prepend=-1.0), np.diff(w, append=10.0))
    k = int(np.argmax(gaps * (f > 1e-3 * f.max())))        # an isolated root with some strength
    eta = 1e-7
    pk = pencil.response_resolvent(A, B, S, sys_.dip, [w[k]], eta)[0]
    assert abs(-eta * pk.imag - f[k] / (2 * w[k])) < 1e-4 * f[k] / (2 * w[k])
    grid = np.linspace(0.2, 3.2, 37)
    np.testing.assert_allclose(pencil.response_from_roots(w, f, grid, 0.02),
                               pencil.response_resolvent(A, B, S, sys_.dip, grid, 0.02), rtol=1e-9, atol=0)
