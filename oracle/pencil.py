"""All eigenpairs of the pencil M z = omega Sigma z, window selection, strengths.

Test infrastructure (see the package docstring): never used by the product.

The generalized eigenvalue equation of the Theory section,
[[A, B], [B, A]] [X; Y] = omega [[S, 0], [0, -S]] [X; Y],
is solved exactly by the textbook symmetric reduction of the RPA problem:

1. L = chol(S); A' = L^-1 A L^-T, B' = L^-1 B L^-T  (metric becomes the identity)
2. C = (A' - B')^(1/2) (symmetric square root by eigh)
3. eigh(C (A' + B') C) = omega^2 T
4. X' + Y' = C T / sqrt(omega), X' - Y' = sqrt(omega) C^-1 T,
   X = L^-T X', Y = L^-T Y'   =>   X^T S X - Y^T S Y = 1 for every root.

Only the positive branch is returned; the negative branch is (-omega, [Y; X]).

Window (reading of the interior-eigenvalue paragraph): the n_roots positive
roots closest to omega0, returned in ascending order; ties within 1e-9 Ha go
to the lower root.

Oscillator strength (reading of the property vector F of the non-diagonal
representation, zeroth order): T^x = sqrt(2) sum_ia mu^x_ia (X + Y)_ia for a
singlet, f = (2/3) omega sum_x (T^x)^2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotStable(RuntimeError):
    """A - B, A + B or S is not positive definite (complex or unphysical roots)."""


def solve_all(A, B, S):
    """All positive roots (ascending) and their S-normalized X, Y (columns)."""
    A = 0.5 * (A + A.T)
    B = 0.5 * (B + B.T)
    S = 0.5 * (S + S.T)
    try:
        L = np.linalg.cholesky(S)
    except np.linalg.LinAlgError as e:
        raise NotStable("S is not positive definite") from e
    Li = sla.solve_triangular(L, np.eye(len(S)), lower=True)
    Ap = Li @ A @ Li.T
    Bp = Li @ B @ Li.T
    wm, Um = np.linalg.eigh(0.5 * ((Ap - Bp) + (Ap - Bp).T))
    if wm.min() <= 0:
        raise NotStable("A - B is not positive definite")
    C = (Um * np.sqrt(wm)) @ Um.T
    Cinv = (Um / np.sqrt(wm)) @ Um.T
    K = C @ (Ap + Bp) @ C
    w2, T = np.linalg.eigh(0.5 * (K + K.T))
    if w2.min() <= 0:
        raise NotStable("A + B is not positive definite")
    omega = np.sqrt(w2)
    XpY = (C @ T) / np.sqrt(omega)
    XmY = (Cinv @ T) * np.sqrt(omega)
    Xt = 0.5 * (XpY + XmY)
    Yt = 0.5 * (XpY - XmY)
    X = sla.solve_triangular(L.T, Xt, lower=False)
    Y = sla.solve_triangular(L.T, Yt, lower=False)
    return omega, X, Y


def select_window(omega, omega0, n_roots):
    """Indices of the n_roots roots nearest omega0 (ties -> lower root), ascending."""
    dist = np.abs(omega - omega0)
    order = np.lexsort((omega, np.round(dist / 1e-9)))
    pick = order[:n_roots]
    return np.sort(pick)


def oscillator_strengths(omega, X, Y, dip, metric=None):
    """f_k = (2/3) omega_k sum_x (sqrt(2) F^x . (X+Y)_k)^2 with the property vector
    F^x = mu^x (zeroth order), or F^x = S mu^x when the metric S is given (the property
    vector over the MP2 ground state through second order); dip is [3][o][v]."""
    mu = dip.reshape(3, -1)
    if metric is not None:
        mu = mu @ metric.T
    T = np.sqrt(2.0) * (mu @ (X + Y))
    return (2.0 / 3.0) * omega * np.sum(T * T, axis=0)


def window_solve(A, B, S, dip, omega0, n_roots, correlated_f=False):
    """Reference result of a window solve: (energies, X, Y, f) for the window."""
    omega, X, Y = solve_all(A, B, S)
    idx = select_window(omega, omega0, n_roots)
    f = oscillator_strengths(omega[idx], X[:, idx], Y[:, idx], dip, S if correlated_f else None)
    return omega[idx], X[:, idx], Y[:, idx], f


def pencil_eigvals_general(M, Sig):
    """Cross-route: all eigenvalues of the general pencil (scipy eig), real parts sorted."""
    w = sla.eig(M, Sig, right=False)
    return np.sort(w.real), np.max(np.abs(w.imag))


def variance(Mop, x):
    """sigma^2(x) = rho_{A^2}(x) - rho_A(x)^2 for a normalized x (error-analysis section)."""
    x = x / np.linalg.norm(x)
    Ax = Mop @ x
    return float(Ax @ Ax - (x @ Ax) ** 2)


def exciton_dos(eps_o, eps_v, dip, edges):
    """Excitonic density of states (Discussion section): per half-open energy bin
    [edges[b], edges[b+1]) the number of particle-hole pairs with eps_a - eps_i inside,
    and the sum of their squared transition dipoles sum_x (mu^x_ia)^2."""
    dE = (eps_v[None, :] - eps_o[:, None]).ravel()
    mu2 = np.sum(dip.reshape(3, -1) ** 2, axis=0) if dip is not None else np.zeros_like(dE)
    counts = np.zeros(len(edges) - 1)
    weights = np.zeros(len(edges) - 1)
    for b in range(len(edges) - 1):
        inside = (dE >= edges[b]) & (dE < edges[b + 1])
        counts[b] = np.count_nonzero(inside)
        weights[b] = mu2[inside].sum()
    return counts, weights


def response_resolvent(A, B, S, dip, omega, eta, F=None):
    """The isotropic polarization propagator of the dipole operator from its non-diagonal
    representation (Theory section, eq. pp_adc): Pi(w) = (1/3) sum_x F_x^T (w Sigma - M)^-1 F_x
    at complex w = omega + i eta, with M = [[A, B], [B, A]], Sigma = diag(S, -S) (the pencil
    of the generalized eigenvalue equation, whose metric the resolvent carries) and the
    property vector F_x = sqrt(2) [mu_x; mu_x] of a singlet excitation (or F given as
    [3][o*v], entering as [F_x; F_x]).  One dense complex solve per frequency, both branches
    at once.  Returns a complex array over omega."""
    N = A.shape[0]
    M = np.block([[A, B], [B, A]]).astype(complex)
    Sig = np.block([[S, np.zeros_like(S)], [np.zeros_like(S), -S]]).astype(complex)
    mu = (dip.reshape(3, -1) if F is None else np.asarray(F).reshape(3, -1))
    Fx = np.sqrt(2.0) * np.concatenate([mu, mu], axis=1).T.astype(complex)   # (2N, 3)
    out = np.empty(len(np.atleast_1d(omega)), dtype=complex)
    for n, w in enumerate(np.atleast_1d(omega)):
        z = complex(w, eta)
        sol = np.linalg.solve(z * Sig - M, Fx)
        out[n] = np.sum(Fx * sol) / 3.0
    assert N == mu.shape[1]
    return out


def response_from_roots(omega_k, f_k, omega, eta):
    """The same propagator summed over the roots of the pencil (its spectral form):
    Pi(w) = sum_k f_k / (2 omega_k) [1 / (w - omega_k) - 1 / (w + omega_k)], w = omega + i eta,
    each positive root with its partner -omega_k on the negative branch."""
    w = np.atleast_1d(omega)[:, None] + 1j * eta
    wk = np.asarray(omega_k)[None, :]
    c = (np.asarray(f_k) / (2.0 * np.asarray(omega_k)))[None, :]
    return np.sum(c * (1.0 / (w - wk) - 1.0 / (w + wk)), axis=1)
