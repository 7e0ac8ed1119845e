"""The interior solver on the CPU, with dense matrix-vector products.

Test infrastructure (see the package docstring): never used by the product.

What comes from the paper (interior-eigenvalue subsection of the Theory section)
and what does not.  The folded target, the inverse-Krylov extension by weighted
Jacobi sweeps and the weight alpha from the folded Rayleigh quotient are the
paper's method, with the readings below where it is silent.  The paired
(X+Y, X-Y) subspace, the 2x2 diagonal corrections from the residuals, the
restarts and the completeness rule are additions of this implementation, shared
with the device solver (they were developed together).  A test that this module
finds the same roots as the full diagonalisation therefore checks that design
against the exact pencil, not an independent rendering of the paper's
algorithm; the device solver is compared with the exact pencil (pencil.py) only.

Steps, with the readings the paper leaves open:

* Target.  The pencil M z = omega Sigma z near a chosen omega0, with
  Z = M - omega0 Sigma (symmetric) and the folded Rayleigh quotient
  rho(y) = |Z y|^2 / |y|^2 = <y|(M - omega0 Sigma)^2|y> / <y|y>.  Its null
  vectors at omega0 = omega_k are the pencil eigenvectors.
* Inverse Krylov basis.  Successive vectors approximate repeated applications
  of the resolvent (M - omega0 Sigma)^-1 to a start block; each application is
  replaced by one weighted Jacobi sweep of Z x = v started from x = v with the
  diagonal/off-diagonal splitting Z = D + F:  x_J = D^-1 (v - F v), hence the
  direction d = x_J - v = D^-1 (v - Z v) and v <- v + alpha d.
* Weight alpha.  The folded Rayleigh quotient of v + alpha d is
  (rho + a1 alpha + a2 alpha^2) / (1 + b1 alpha + b2 alpha^2) for unit v with
  a1 = 2 (Zv).(Zd), a2 = |Zd|^2, b1 = 2 v.d, b2 = |d|^2; alpha is the
  stationary point with the smaller quotient, or 1 if none is real.  Z is
  linear, so Z(v + alpha d) = Zv + alpha Zd: one product per step.
* Subspace.  Every 2N-vector [X; Y] that enters contributes its two halves to
  an orthonormal basis Q of the N-dimensional particle-hole space (a "paired"
  subspace: it holds [X; Y] and its partner [Y; X]), by classical Gram-Schmidt
  applied twice.  The products (A+B)Q, (A-B)Q and SQ follow the same linear
  transforms, so orthonormalization costs no extra products.
* Extraction.  The projected problem keeps the exact block structure of the
  pencil (A+B and A-B positive definite, S positive definite), so its
  eigenvalues are real and come in +-theta pairs; it is solved exactly by the
  same symmetric reduction as the full problem.  Reading of the folded
  criterion: among the positive Ritz pairs the window takes the n_roots with
  the smallest folded Rayleigh quotient at omega0; energies are pencil Ritz
  values (not folded Ritz values, which differ from (omega - omega0)^2 when
  B is nonzero).
* Restart and refinement.  Residuals r = (M - theta Sigma) y of the Ritz
  pairs are turned into corrections by the diagonal of the shifted pencil
  (a 2x2 solve per particle-hole pair in the (X+Y, X-Y) coordinates); they
  start the next cycle's Jacobi steps.  When the basis is full it is replaced
  by the X+Y and X-Y parts of the block's Ritz vectors.
* Completeness (the paper does not say when a window is finished).  Ritz
  extraction is unreliable for interior eigenvalues: an eigenvector that is
  almost entirely in the subspace can appear as a polluted Ritz pair next to
  omega0 with a large residual and a large folded quotient, and spurious Ritz
  values appear there too.  So the window is converged only when every Ritz
  pair whose value lies within the farthest target's distance of omega0 has
  |r| <= tol |y|; those pairs lead the block, so they are corrected and kept
  at restarts, and the result is the n_roots of them nearest omega0.
"""
from __future__ import annotations

import numpy as np

from . import pencil


def alpha_weight(rho, a1, a2, b1, b2):
    """Stationary point of (rho + a1 x + a2 x^2) / (1 + b1 x + b2 x^2) with the smaller value."""
    qa = a2 * b1 - a1 * b2
    qb = 2.0 * (a2 - rho * b2)
    qc = a1 - rho * b1
    cands = []
    scale = max(abs(qa), abs(qb), abs(qc), 1e-300)
    if abs(qa) <= 1e-14 * scale:
        if abs(qb) > 0:
            cands.append(-qc / qb)
    else:
        disc = qb * qb - 4 * qa * qc
        if disc >= 0:
            s = np.sqrt(disc)
            q = -0.5 * (qb + np.copysign(s, qb))
            if q != 0:
                cands += [q / qa, qc / q]
            else:
                cands.append(-qb / (2 * qa))
    best, best_val = 1.0, None
    for x in cands:
        den = 1 + b1 * x + b2 * x * x
        if den <= 0:
            continue
        val = (rho + a1 * x + a2 * x * x) / den
        if best_val is None or val < best_val:
            best, best_val = x, val
    return best


class _Ops:
    """Dense A, B, S with a product counter (one count per particle-hole vector)."""

    def __init__(self, A, B, S):
        self.A, self.B, self.S = A, B, S
        self.count = 0

    def apply(self, V):
        """(A+B)V, (A-B)V, SV."""
        self.count += V.shape[1]
        AV, BV = self.A @ V, self.B @ V
        return AV + BV, AV - BV, self.S @ V


def _orthonormalize(Q, V, drop=1e-12):
    """CGS2 of V against orthonormal Q, then symmetric orthonormalization.

    Returns (Vn, C, R) with V ~= Q C + Vn R and Vn orthonormal and orthogonal
    to Q.  Directions with squared norm below drop after the first projection
    (relative to the column's norm), or that lose more than half their norm in
    the second projection, are numerically in span(Q) and are not returned.
    """
    nb, k = Q.shape[1], V.shape[1]

    def project(V):
        if nb:
            C = Q.T @ V
            return V - Q @ C, C
        return V, np.zeros((0, V.shape[1]))

    def sym_orth(V, thresh):
        G = V.T @ V
        lam, U = np.linalg.eigh(0.5 * (G + G.T))
        keep = lam > thresh
        T = U[:, keep] / np.sqrt(lam[keep])
        R = (U[:, keep] * np.sqrt(lam[keep])).T
        return V @ T, R

    nrm = np.linalg.norm(V, axis=0)
    nrm = np.where(nrm > 0, nrm, 1.0)
    V1, C1 = project(V / nrm)
    V2, R1 = sym_orth(V1, drop)
    V3, C2 = project(V2)
    V4, R2 = sym_orth(V3, 0.25)
    C = (C1 + C2 @ R1) * nrm
    R = (R2 @ R1) * nrm
    return V4, C, R


def folded_window_solve(A, B, S, omega0, n_roots, *, block=None, krylov_steps=2, max_basis=None,
                        tol=1e-9, max_cycles=100, d_clamp=1e-4, seed=0):
    """Paper's interior solver on dense A, B, S.

    Returns (theta, X, Y, info): the n_roots window roots (ascending), their
    S-normalized eigenvectors (columns, X^T S X - Y^T S Y = 1) and statistics.
    Block vectors are kept as coefficients in the basis Q; every product is a
    linear combination of the stored (A+B)Q, (A-B)Q and SQ.
    """
    N = A.shape[0]
    m = min(block or (n_roots + 2), N)
    nb_max = min(max_basis or max(480, 20 * m), N)
    ops = _Ops(A, B, S)
    dA, dB, dS = np.diag(A).copy(), np.diag(B).copy(), np.diag(S).copy()

    def clamp(x):
        return np.where(np.abs(x) < d_clamp, np.where(x >= 0, d_clamp, -d_clamp), x)

    Dtop = clamp(dA - omega0 * dS)
    Dbot = clamp(dA + omega0 * dS)

    Q = np.zeros((N, 0))
    P = [np.zeros((N, 0)) for _ in range(3)]          # (A+B)Q, (A-B)Q, SQ

    def extend(V):
        """Add span(V) to the basis; return coefficients of V in the new basis."""
        nonlocal Q, P
        Vn, C, R = _orthonormalize(Q, V)
        if Vn.shape[1]:
            Pn = ops.apply(Vn)
            Q = np.hstack([Q, Vn])
            P = [np.hstack([p, pn]) for p, pn in zip(P, Pn)]
        return np.vstack([C, R])

    def pad(c):
        return np.vstack([c, np.zeros((Q.shape[1] - c.shape[0], c.shape[1]))])

    def zprod(cx, cy):
        """Z [X; Y] for X = Q cx, Y = Q cy: top = A X + B Y - w0 S X, bottom = B X + A Y + w0 S Y."""
        cu, cw = cx + cy, cx - cy
        PU, MW = P[0] @ cu, P[1] @ cw
        SX, SY = P[2] @ cx, P[2] @ cy
        return 0.5 * (PU + MW) - omega0 * SX, 0.5 * (PU - MW) + omega0 * SY

    rng = np.random.default_rng(seed)
    start = np.argsort(np.abs(Dtop), kind="stable")[:m]
    X0 = np.zeros((N, m))
    X0[start, np.arange(m)] = 1.0
    X0 += 1e-3 * rng.standard_normal((N, m))
    Y0 = 1e-3 * rng.standard_normal((N, m))
    newX, newY = X0, Y0

    info = dict(cycles=0, products=0, converged=False)
    for cycle in range(max_cycles):
        c = extend(np.hstack([newX, newY]))
        k = newX.shape[1]
        cx, cy = c[:, :k], c[:, k:]
        for s in range(1, krylov_steps):
            if Q.shape[1] + 2 * k > nb_max:
                break
            # weighted-Jacobi step on each 2N column z = [X; Y] = [Q cx; Q cy]
            nz = np.sqrt(np.sum(cx * cx, 0) + np.sum(cy * cy, 0))
            cx, cy = cx / nz, cy / nz
            Zt, Zb = zprod(cx, cy)
            dX = (Q @ cx - Zt) / Dtop[:, None]
            dY = (Q @ cy - Zb) / Dbot[:, None]
            cd = extend(np.hstack([dX, dY]))
            cx, cy = pad(cx), pad(cy)
            Zt, Zb = zprod(cx, cy)
            cdx, cdy = cd[:, :k], cd[:, k:]
            Zdt, Zdb = zprod(cdx, cdy)
            for j in range(k):
                rho = Zt[:, j] @ Zt[:, j] + Zb[:, j] @ Zb[:, j]
                a1 = 2 * (Zt[:, j] @ Zdt[:, j] + Zb[:, j] @ Zdb[:, j])
                a2 = Zdt[:, j] @ Zdt[:, j] + Zdb[:, j] @ Zdb[:, j]
                b1 = 2 * (cx[:, j] @ cdx[:, j] + cy[:, j] @ cdy[:, j])
                b2 = cdx[:, j] @ cdx[:, j] + cdy[:, j] @ cdy[:, j]
                al = alpha_weight(rho, a1, a2, b1, b2)
                cx[:, j] += al * cdx[:, j]
                cy[:, j] += al * cdy[:, j]
        # pencil Rayleigh-Ritz in the paired subspace (exact small RPA problem)
        Ap = Q.T @ P[0]
        Am = Q.T @ P[1]
        Sp = Q.T @ P[2]
        th, Xs, Ys = pencil.solve_all(0.5 * (Ap + Am), 0.5 * (Ap - Am), Sp)
        us, ws = Xs + Ys, Xs - Ys
        PU, MW = P[0] @ us, P[1] @ ws
        SU, SW = P[2] @ us, P[2] @ ws
        # residuals of the pencil in (u, w) coordinates and folded quotient at omega0
        ru = PU - th * SW
        rw = MW - th * SU
        ynorm = np.sqrt(0.5 * (np.sum(us * us, 0) + np.sum(ws * ws, 0)))
        rnorm = np.sqrt(0.5 * (np.sum(ru * ru, 0) + np.sum(rw * rw, 0))) / ynorm
        fu = PU - omega0 * SW
        fw = MW - omega0 * SU
        folded = 0.5 * (np.sum(fu * fu, 0) + np.sum(fw * fw, 0)) / ynorm ** 2
        order = np.argsort(folded, kind="stable")
        tgt = order[:n_roots]
        # every Ritz value within the farthest target's distance of omega0 must
        # converge as well; those pairs lead the block (see the module docstring)
        dmax = np.abs(th[tgt] - omega0).max()
        inner = np.where(np.abs(th - omega0) <= dmax * (1 + 1e-12))[0]
        inner = inner[np.argsort(np.abs(th[inner] - omega0), kind="stable")]
        blk = list(inner[:m])
        for j in order:
            if len(blk) >= m:
                break
            if j not in blk:
                blk.append(j)
        blk = np.array(blk)
        out = inner[:n_roots] if len(inner) >= n_roots else tgt
        info.update(cycles=cycle + 1, products=ops.count, basis=Q.shape[1])
        sel = out[np.argsort(th[out])]
        result = (th[sel], Q @ Xs[:, sel], Q @ Ys[:, sel])
        info["residuals"] = rnorm[sel]
        if np.all(rnorm[tgt] <= tol) and np.all(rnorm[inner] <= tol):
            info["converged"] = True
            break
        # corrections: diagonal of the shifted pencil in (u, w) coordinates
        ap = (dA + dB)[:, None]
        am = (dA - dB)[:, None]
        s_ = dS[:, None]
        act = blk[rnorm[blk] > tol]
        thb = th[act][None, :]
        det = clamp(ap * am - thb * thb * s_ * s_)
        cu_ = -(am * ru[:, act] + thb * s_ * rw[:, act]) / det
        cw_ = -(thb * s_ * ru[:, act] + ap * rw[:, act]) / det
        newX = 0.5 * (cu_ + cw_)
        newY = 0.5 * (cu_ - cw_)
        if Q.shape[1] + 2 * krylov_steps * len(act) > nb_max:
            # thick restart: orthonormal basis of the block's Ritz halves (X+Y, X-Y)
            K, _ = np.linalg.qr(np.hstack([us[:, blk], ws[:, blk]]))
            Q = Q @ K
            P = [p @ K for p in P]
    return result + (info,)
