"""Closed-shell singlet A, B, S matrices, assembled densely in FP64.

Test infrastructure (see the package docstring): never used by the product.

What is assembled (Theory section, "Second-order approximation of the
polarization propagator"): the response matrix M = [[A, B], [B, A]] with metric
Sigma = diag(S, -S) (the generalized eigenvalue equation of that section), each
block written as a sum of zeroth, first and second order parts.

Readings of the paper (each is listed with its justification in the design
notes of the repository):

* Orbital basis: real, closed-shell, spin-adapted to singlets.  Compound index
  ia = i*v + a (occupied-major, matching the [o][v] layout of the C ABI).
* Integrals: chemists' notation (pq|rs) = sum_P B_Ppq B_Prs (density fitting,
  Results section).
* A0 = (eps_a - eps_i) delta delta, S0 = delta delta, B0 = 0, S1 = 0 (equations
  for the zeroth/first order overlap and A, B).
* A1 and B1 are the antisymmetrized two-electron elements of the first-order
  equations, i.e. singlet TDHF: A1 = 2(ia|jb) - (ij|ab), B1 = 2(ia|jb) - (ib|ja),
  with the sign of B fixed so that the transition vector is X + Y (the text
  identifies first order with CIS/TDHF).
* Second order: the defining expectation values over the MP2 ground state
  |0> + R0 W_N |0> (only doubles, as the paper states), expanded consistently to
  second order in W_N, with the symmetrized double commutator for A.  The
  resulting closed forms below are not printed in the paper; they are pinned
  against a brute-force Fock-space evaluation of the definitions
  (oracle.fockspace) and against the spin-orbital route (oracle.spinorb).
"""
from __future__ import annotations

import numpy as np


def _full_B(sys):
    """Full symmetric DF factors B[P, p, q] over all o+v orbitals (occupied first)."""
    o, v, naux = sys.o, sys.v, sys.naux
    n = o + v
    B = np.zeros((naux, n, n))
    B[:, :o, :o] = sys.B_oo
    B[:, :o, o:] = sys.B_ov
    B[:, o:, :o] = np.transpose(sys.B_ov, (0, 2, 1))
    B[:, o:, o:] = sys.B_vv
    return B


def eri_ovov(sys):
    """(ia|jb) as a 4-index array [i, a, j, b]."""
    o, v, naux = sys.o, sys.v, sys.naux
    L = sys.B_ov.reshape(naux, o * v)
    return (L.T @ L).reshape(o, v, o, v)


def eri_oovv(sys):
    """(ij|ab) as [i, j, a, b]."""
    o, v, naux = sys.o, sys.v, sys.naux
    return (sys.B_oo.reshape(naux, o * o).T @ sys.B_vv.reshape(naux, v * v)).reshape(o, o, v, v)


def eri_oooo(sys):
    """(ij|kl) as [i, j, k, l]."""
    o, naux = sys.o, sys.naux
    L = sys.B_oo.reshape(naux, o * o)
    return (L.T @ L).reshape(o, o, o, o)


def eri_vvvv(sys):
    """(ab|cd) as [a, b, c, d] (v^4 storage: small systems only)."""
    v, naux = sys.v, sys.naux
    L = sys.B_vv.reshape(naux, v * v)
    return (L.T @ L).reshape(v, v, v, v)


def eri_ovvv(sys):
    """(ia|bc) as [i, a, b, c]."""
    o, v, naux = sys.o, sys.v, sys.naux
    return (sys.B_ov.reshape(naux, o * v).T @ sys.B_vv.reshape(naux, v * v)).reshape(o, v, v, v)


def eri_ovoo(sys):
    """(ia|jk) as [i, a, j, k]."""
    o, v, naux = sys.o, sys.v, sys.naux
    return (sys.B_ov.reshape(naux, o * v).T @ sys.B_oo.reshape(naux, o * o)).reshape(o, v, o, o)


def denominators(sys):
    """D[i, j, a, b] = eps_i + eps_j - eps_a - eps_b."""
    eo, ev = sys.eps_o, sys.eps_v
    return eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]


def mp2_amplitudes(sys):
    """Closed-shell first-order amplitudes t[i,j,a,b] = (ia|jb) / D_ij^ab.

    Spatial-orbital form of R0 W_N |0> (the 2p2h-only first-order correction in
    the MP2 paragraph of the Theory section).
    """
    ovov = eri_ovov(sys)
    return np.transpose(ovov, (0, 2, 1, 3)) / denominators(sys)


def tau_amplitudes(t):
    """tau[i,j,a,b] = 2 t[i,j,a,b] - t[i,j,b,a] (singlet-coupled amplitudes)."""
    return 2.0 * t - np.transpose(t, (0, 1, 3, 2))


def mp2_energy(sys):
    """E(2) = sum_ijab tau_ij^ab (ia|jb): the closed-shell MP2 correlation energy."""
    t = mp2_amplitudes(sys)
    ovov = eri_ovov(sys)
    return float(np.einsum("ijab,iajb->", tau_amplitudes(t), ovov))


def second_order_intermediates(sys):
    """The vv/oo intermediates of the second-order metric and A block.

    Gv[a,b] = sum_kld tau_kl^ad t_kl^bd            (virtual MP2 occupation)
    Ev[a,b] = sum_kld tau_kl^ad t_kl^bd (eps_k + eps_l - eps_d)
    Go[i,j] = sum_kcd tau_ik^cd t_jk^cd            (occupied MP2 depletion)
    Eo[i,j] = sum_kcd tau_ik^cd t_jk^cd (eps_k - eps_c - eps_d)
    """
    eo, ev = sys.eps_o, sys.eps_v
    t = mp2_amplitudes(sys)
    tau = tau_amplitudes(t)
    Gv = np.einsum("klad,klbd->ab", tau, t)
    w_v = eo[:, None, None] + eo[None, :, None] - ev[None, None, :]          # [k,l,d]
    Ev = np.einsum("klad,klbd,kld->ab", tau, t, w_v)
    Go = np.einsum("ikcd,jkcd->ij", tau, t)
    w_o = eo[:, None, None] - ev[None, :, None] - ev[None, None, :]         # [k,c,d]
    Eo = np.einsum("ikcd,jkcd,kcd->ij", tau, t, w_o)
    return dict(Gv=Gv, Ev=Ev, Go=Go, Eo=Eo, t=t, tau=tau)


def assemble(sys, order: int):
    """Return (A, B, S) as N x N arrays (N = o*v, index ia = i*v + a).

    order 0: A = Delta, B = 0, S = 1 (the Hartree-Fock spectrum of the Results
    section); order 1: adds the TDHF two-electron terms; order 2: adds the MP2
    corrections S2, A2, B2.
    """
    if order not in (0, 1, 2):
        raise ValueError("order must be 0, 1 or 2")
    o, v = sys.o, sys.v
    N = o * v
    eo, ev = sys.eps_o, sys.eps_v
    dI = np.eye(o)
    dA = np.eye(v)
    delta_ia = (ev[None, :] - eo[:, None]).reshape(N)
    A = np.diag(delta_ia).astype(float)
    B = np.zeros((N, N))
    S = np.eye(N)
    if order == 0:
        return A, B, S

    ovov = eri_ovov(sys)                              # (ia|jb)
    oovv = eri_oovv(sys)                              # (ij|ab)
    J = ovov                                           # [i,a,j,b]
    K_A = np.transpose(oovv, (0, 2, 1, 3))            # (ij|ab) -> [i,a,j,b]
    K_B = np.transpose(ovov, (0, 3, 2, 1))            # (ib|ja) -> [i,a,j,b]
    A = A + (2.0 * J - K_A).reshape(N, N)
    B = B + (2.0 * J - K_B).reshape(N, N)
    if order == 1:
        return A, B, S

    it = second_order_intermediates(sys)
    Gv, Ev, Go, Eo, tau = it["Gv"], it["Ev"], it["Go"], it["Eo"], it["tau"]

    # S2_{ia,jb} = -delta_ab Go_ij - delta_ij Gv_ab
    S2 = -np.einsum("ij,ab->iajb", Go, dA) - np.einsum("ij,ab->iajb", dI, Gv)
    # A2_{ia,jb} = -delta_ij (Ev_ab - eps_i Gv_ab) - delta_ab (eps_a Go_ij + Eo_ij)
    A2 = (-np.einsum("ij,ab->iajb", dI, Ev)
          + np.einsum("i,ij,ab->iajb", eo, dI, Gv)
          - np.einsum("a,ij,ab->iajb", ev, Go, dA)
          - np.einsum("ij,ab->iajb", Eo, dA))
    B2 = b2_dense(sys, tau)
    A = A + A2.reshape(N, N)
    S = S + S2.reshape(N, N)
    B = B + B2.reshape(N, N)
    return A, B, S


def b2_dense(sys, tau, ladder: str = "auto"):
    """Second-order B block, element form, [i,a,j,b].

    B2_{ia,jb} = sum_cd (ac|bd) tau_ij^cd            pp ladder
               + sum_kl (ki|lj) tau_kl^ab            hh ladder
               - sum_kc (ki|bc) tau_kj^ac            ring (exchange-type)
               - sum_kc (kj|ac) tau_ik^cb            ring (exchange-type)
               - sum_kc (kc|bi) tau_jk^ac            ring (Coulomb-type)
               - sum_kc (kc|aj) tau_ik^bc            ring (Coulomb-type)

    The pp ladder is taken either through the (ac|bd) array ("eri", v^4 storage) or
    factor by factor, sum_P B_P,ac tau_ij^cd B_P,bd ("per_P", for large v); "auto"
    chooses by the size of (ac|bd).
    """
    o, v, naux = sys.o, sys.v, sys.naux
    if ladder not in ("auto", "eri", "per_P"):
        raise ValueError("ladder must be 'auto', 'eri' or 'per_P'")
    # pp ladder via the DF factors: sum_P (B_P tau_ij B_P)_ab
    if ladder == "eri" or (ladder == "auto" and v ** 4 * 8 <= 6e9):
        vvvv = eri_vvvv(sys)                                        # (ac|bd) = [a,c,b,d]
        ladder_pp = np.einsum("acbd,ijcd->iajb", vvvv, tau, optimize=True)
    else:
        ladder_pp = np.zeros((o, v, o, v))
        for P in range(naux):
            Bp = sys.B_vv[P]
            ladder_pp += np.einsum("ac,ijcd,bd->iajb", Bp, tau, Bp, optimize=True)
    oooo = eri_oooo(sys)                                            # (ki|lj) = [k,i,l,j]
    ladder_hh = np.einsum("kilj,klab->iajb", oooo, tau, optimize=True)
    oovv = eri_oovv(sys)                                            # (ki|bc) = [k,i,b,c]
    ring_k1 = -np.einsum("kibc,kjac->iajb", oovv, tau, optimize=True)
    ring_k2 = -np.einsum("kjac,ikcb->iajb", oovv, tau, optimize=True)
    ovov = eri_ovov(sys)                                            # (kc|bi) = (ib|kc) = [i,b,k,c]
    ring_j1 = -np.einsum("ibkc,jkac->iajb", ovov, tau, optimize=True)
    ring_j2 = -np.einsum("jakc,ikbc->iajb", ovov, tau, optimize=True)
    return ladder_pp + ladder_hh + ring_k1 + ring_k2 + ring_j1 + ring_j2


def build_M(sys, order: int):
    """M = [[A, B], [B, A]] and Sigma = diag(S, -S), both 2N x 2N."""
    A, B, S = assemble(sys, order)
    M = np.block([[A, B], [B, A]])
    Z = np.zeros_like(S)
    Sig = np.block([[S, Z], [Z, -S]])
    return M, Sig


def sigma_dense(sys, order: int, Xblk, metric: bool = False):
    """Reference product for the C ABI: Xblk is [m][2][o*v] ([X;Y] per vector).

    Returns M @ [X;Y] per vector (or Sigma @ [X;Y] if metric), same layout.
    """
    A, B, S = assemble(sys, order)
    X = Xblk[:, 0, :].T
    Y = Xblk[:, 1, :].T
    if metric:
        top, bot = S @ X, -(S @ Y)
    else:
        top, bot = A @ X + B @ Y, B @ X + A @ Y
    return np.stack([top.T, bot.T], axis=1)


def diag_M(sys, order: int):
    """Diagonals of A and S (the D of the Jacobi splitting is built from them)."""
    A, _, S = assemble(sys, order)
    return np.diag(A).copy(), np.diag(S).copy()
