"""Riesz projector of the pencil M z = omega Sigma z on a circular contour, and a window
solve by contour-filtered subspace iteration.

Test infrastructure (see the package docstring): never used by the product.

The section on the connection to the Riesz projector defines, for a closed contour
Gamma in the complex plane, P = (1 / 2 pi i) closed-integral over Gamma of (z I - M)^-1 dz;
applied to a vector it keeps the part of the vector in the eigenspace of the eigenvalues
enclosed by Gamma.  For the generalized problem of the Theory section (metric Sigma) the
same operator reads

    P = (1 / 2 pi i) closed-integral (z Sigma - M)^-1 Sigma dz,

because (z Sigma - M)^-1 Sigma z_k = z_k / (z - omega_k) for every eigenpair
M z_k = omega_k Sigma z_k (the residue at omega_k is z_k).

Readings (listed in the design notes):

* Contour: the circle of center c (real) and radius r.
* Quadrature: trapezoidal rule with 2n equally spaced nodes z_k = c + r e^{i theta_k},
  theta_k = pi (2k + 1) / (2n), none on the real axis.  M, Sigma and the vectors are
  real, so the node in the lower half plane gives the complex conjugate of its mirror
  node's term, and
      P v = (1/n) sum_{k < n} Re( r e^{i theta_k} (z_k Sigma - M)^-1 Sigma v ).
* Filter: on an eigenvector with eigenvalue omega the rule gives rho(x) z_k,
  x = (omega - c) / r, rho(x) = 1 / (1 + x^(2n)).  (The nodes e^{i theta_k} are the
  roots of u^(2n) = -1, and (1/2n) sum_k u_k / (u_k - x) is the partial-fraction
  expansion of 1 / (1 + x^(2n)).)  rho is close to 1 inside the circle and decays as
  |x|^(-2n) outside.
* Window solve (the projector used in place of the folded-spectrum steps): subspace
  iteration Q <- P Q with a Rayleigh-Ritz step of the pencil on span(Q) after each
  application, until the n_roots Ritz pairs nearest omega0 have residual
  |(M - theta Sigma) y| / |y| <= tol.  The circle is re-centred at omega0 and its radius
  placed halfway between the n_roots-th and the next Ritz value (by distance to
  omega0), so that the window's roots are inside and the rest outside.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pencil_matrices(A, B, S):
    """M = [[A, B], [B, A]] and Sigma = diag(S, -S)."""
    Z = np.zeros_like(S)
    return np.block([[A, B], [B, A]]), np.block([[S, Z], [Z, -S]])


def contour_nodes(c, r, n):
    """The n nodes of the upper half circle and their weights r e^{i theta_k} / n."""
    theta = np.pi * (2 * np.arange(n) + 1) / (2 * n)
    u = np.exp(1j * theta)
    return c + r * u, r * u / n


def filter_value(x, n):
    """rho(x) = 1 / (1 + x^(2n)) of the 2n-node trapezoidal rule (x = (omega - c) / r)."""
    x = np.asarray(x, dtype=float)
    return 1.0 / (1.0 + x ** (2 * n))


def riesz_apply(M, Sig, V, c, r, n):
    """P V for real V (columns), each shifted system solved exactly (dense LU)."""
    z, w = contour_nodes(c, r, n)
    rhs = Sig @ V
    out = np.zeros(V.shape)
    for zk, wk in zip(z, w):
        out += np.real(wk * np.linalg.solve(zk * Sig - M, rhs.astype(complex)))
    return out


def _rayleigh_ritz(M, Sig, Q):
    """Positive-branch Ritz pairs of the pencil on span(Q): M is positive definite, so
    (Q^T Sigma Q) c = mu (Q^T M Q) c is a definite symmetric problem with mu = 1/omega."""
    Q, _ = np.linalg.qr(Q)
    Mp = Q.T @ M @ Q
    Sp = Q.T @ Sig @ Q
    mu, C = sla.eigh(0.5 * (Sp + Sp.T), 0.5 * (Mp + Mp.T))
    pos = mu > 0
    theta = 1.0 / mu[pos]
    Y = Q @ C[:, pos]
    return theta, Y


def riesz_window_solve(A, B, S, omega0, n_roots, *, nodes=8, m0=None, tol=1e-10, max_iter=60, seed=0):
    """Window solve by contour-filtered subspace iteration (dense, exact shifted solves).

    Returns (energies ascending, X, Y, iterations) with X^T S X - Y^T S Y = 1 per root."""
    M, Sig = pencil_matrices(A, B, S)
    N = A.shape[0]
    m0 = m0 or min(2 * N, 2 * n_roots + 4)
    # start: the zeroth-order picture (diagonal estimates) sets the first circle
    est = np.diag(A) / np.diag(S)
    d = np.sort(np.abs(est - omega0))
    r = 1.5 * d[min(n_roots, N) - 1] + 1e-6
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((2 * N, m0))
    for it in range(1, max_iter + 1):
        Q = riesz_apply(M, Sig, Q, omega0, r, nodes)
        theta, Y = _rayleigh_ritz(M, Sig, Q)
        order = np.argsort(np.abs(theta - omega0), kind="stable")
        pick = order[:n_roots]
        res = []
        for j in pick:
            y = Y[:, j]
            res.append(np.linalg.norm(M @ y - theta[j] * (Sig @ y)) / np.linalg.norm(y))
        if len(pick) == n_roots and max(res) <= tol:
            break
        dist = np.abs(theta[order] - omega0)
        if len(dist) > n_roots:
            r = 0.5 * (dist[n_roots - 1] + dist[n_roots])
        Q = Y
    idx = pick[np.argsort(theta[pick])]
    Z = Y[:, idx]
    # Sigma-normalise (positive branch: z^T Sigma z > 0)
    nrm = np.einsum("ik,ik->k", Z, Sig @ Z)
    Z = Z / np.sqrt(nrm)
    return theta[idx], Z[:N], Z[N:], it
