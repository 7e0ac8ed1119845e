"""Exact single rows of the zeroth+first-order A and B blocks at any size.

Test infrastructure (see the package docstring): never used by the product.

Where the dense matrices cannot be formed (particle-hole dimension 1.6e5 and
more), sampled rows of the first-order blocks are still cheap to evaluate from
their definitions (Theory section: the zeroth-order diagonal of eq. a(0) and
the first-order elements of eqs. a(1), b(1), read as singlet TDHF):

    A_{ia,jb} = (eps_a - eps_i) delta_ij delta_ab + 2 (ia|jb) - (ij|ab)
    B_{ia,jb} = 2 (ia|jb) - (ib|ja)

with (pq|rs) = sum_P B_Ppq B_Prs (density fitting).  Row ia needs B_ov in full,
the slice B_oo[:, i, :] and the slice B_vv[:, a, :]; each row costs
O(naux * o * v).
"""
from __future__ import annotations

import numpy as np


def first_order_rows(eps, o, v, B_ov, rows, Boo_i, Bvv_a, V):
    """(A V)[q, ia] and (B V)[q, ia] for the sampled compound indices 'rows'.

    eps   : (o+v,) orbital energies, occupied first
    B_ov  : (naux, o, v)
    rows  : list of compound indices ia = i*v + a
    Boo_i : list, Boo_i[t] = B_oo[:, i_t, :]  (naux, o)
    Bvv_a : list, Bvv_a[t] = B_vv[:, a_t, :]  (naux, v)
    V     : (k, o*v) particle-hole vectors
    Returns (AV, BV), each (k, len(rows)).
    """
    naux = B_ov.shape[0]
    L = B_ov.reshape(naux, o * v)
    k = V.shape[0]
    AV = np.zeros((k, len(rows)))
    BV = np.zeros((k, len(rows)))
    iajb_rows = L[:, list(rows)].T @ L                       # (ia|jb) for every sampled ia
    for t, ia in enumerate(rows):
        i, a = divmod(int(ia), v)
        iajb = iajb_rows[t]
        ijab = (np.ascontiguousarray(Boo_i[t]).T @ np.ascontiguousarray(Bvv_a[t])).reshape(o * v)  # (ij|ab): [j][b]
        ibja = (np.ascontiguousarray(B_ov[:, :, a]).T @ np.ascontiguousarray(B_ov[:, i, :])).reshape(o * v)  # (ib|ja)
        a_row = 2.0 * iajb - ijab
        b_row = 2.0 * iajb - ibja
        a_row[ia] += eps[o + a] - eps[i]
        AV[:, t] = V @ a_row
        BV[:, t] = V @ b_row
    return AV, BV


# ---------------------------------------------------------------------------
# Second order.  Element form of the singlet second-order blocks (Theory section,
# "Second-order approximation": eqs. s(2), a(2), b(2) expanded over the MP2 ground
# state; the same expressions dense.assemble writes out for whole matrices):
#
#   B2_{ia,jb} = sum_cd (ac|bd) tau_ij^cd + sum_kl (ki|lj) tau_kl^ab
#              - sum_kc (ki|bc) tau_kj^ac - sum_kc (kj|ac) tau_ik^cb
#              - sum_kc (kc|bi) tau_jk^ac - sum_kc (kc|aj) tau_ik^bc
#   A2_{ia,jb} = -delta_ij (Ev_ab - eps_i Gv_ab) - delta_ab (eps_a Go_ij + Eo_ij)
#   S2_{ia,jb} = -delta_ab Go_ij - delta_ij Gv_ab
#
# with t_ij^ab = (ia|jb) / (eps_i + eps_j - eps_a - eps_b), tau_ij^ab = 2 t_ij^ab - t_ij^ba
# and the MP2 densities Gv, Ev, Go, Eo of dense.second_order_intermediates.  A row ia of
# B2 needs the amplitudes with first occupied index i (tau_i[j][c][d] = tau_ij^cd) and
# those with first virtual index a (tau^a[k][l][d] = tau_kl^ad), plus integral slices
# for i and a; no o^2 v^2 array is formed.


def _amplitudes_i(eps, o, v, L, i):
    """tau_i[j, c, d] = tau_ij^cd for one occupied i (L = B_ov as [naux][o*v]); also
    returns (ic|jd) as [c, j, d]."""
    eo, ev = eps[:o], eps[o:]
    naux = L.shape[0]
    icjd = (np.ascontiguousarray(L.reshape(naux, o, v)[:, i, :]).T @ L).reshape(v, o, v)          # (ic|jd) [c][j][d]
    D = (eo[i] + eo[:, None, None] - ev[None, :, None] - ev[None, None, :])  # [j][c][d]
    t = np.transpose(icjd, (1, 0, 2)) / D                                    # t_ij^cd [j][c][d]
    return 2.0 * t - np.transpose(t, (0, 2, 1)), icjd


def _amplitudes_a(eps, o, v, L, a):
    """tau^a[k, l, d] = tau_kl^ad for one virtual a; also returns (ka|ld) as [k, l, d]."""
    eo, ev = eps[:o], eps[o:]
    naux = L.shape[0]
    kald = (np.ascontiguousarray(L.reshape(naux, o, v)[:, :, a]).T @ L).reshape(o, o, v)          # (ka|ld) [k][l][d]
    D = eo[:, None, None] + eo[None, :, None] - ev[a] - ev[None, None, :]
    t = kald / D                                                              # t_kl^ad
    return 2.0 * t - np.transpose(t, (1, 0, 2)), kald                         # t_kl^da = t_lk^ad


def b2_row(eps, o, v, B_oo, B_ov, B_vv, ia):
    """Row ia of the second-order B block, B2[ia, jb] as an (o, v) array."""
    naux = B_ov.shape[0]
    i, a = divmod(int(ia), v)
    L = B_ov.reshape(naux, o * v)
    tau_i, icjd = _amplitudes_i(eps, o, v, L, i)          # [j][c][d], (ic|jd) [c][j][d]
    tau_a, kald = _amplitudes_a(eps, o, v, L, a)          # [k][l][d], (ka|ld) [k][l][d]
    Boo_i = np.ascontiguousarray(B_oo[:, :, i])           # B_P,ki  [P][k]
    # sum_cd (ac|bd) tau_ij^cd
    acbd = (np.ascontiguousarray(B_vv[:, a, :]).T @ B_vv.reshape(naux, v * v)).reshape(v, v, v)        # [c][b][d]
    row = np.einsum("cbd,jcd->jb", acbd, tau_i, optimize=True)
    del acbd
    # + sum_kl (ki|lj) tau_kl^ab
    kilj = (Boo_i.T @ B_oo.reshape(naux, o * o)).reshape(o, o, o)               # [k][l][j]
    row += np.einsum("klj,klb->jb", kilj, tau_a, optimize=True)
    # - sum_kc (ki|bc) tau_kj^ac
    kibc = (Boo_i.T @ B_vv.reshape(naux, v * v)).reshape(o, v, v)               # [k][b][c]
    row -= np.einsum("kbc,kjc->jb", kibc, tau_a, optimize=True)
    del kibc
    # - sum_kc (kj|ac) tau_ik^cb
    kjac = (B_oo.reshape(naux, o * o).T @ np.ascontiguousarray(B_vv[:, a, :])).reshape(o, o, v)        # [k][j][c]
    row -= np.einsum("kjc,kcb->jb", kjac, tau_i, optimize=True)
    # - sum_kc (kc|bi) tau_jk^ac = - sum_kc (ib|kc) tau^a[j][k][c]
    row -= np.einsum("bkc,jkc->jb", icjd, tau_a, optimize=True)
    # - sum_kc (kc|aj) tau_ik^bc = - sum_kc (ja|kc) tau_i[k][b][c]
    row -= np.einsum("jkc,kbc->jb", kald, tau_i, optimize=True)                 # (ja|kc) = kald[j][k][c]
    return row


def mp2_densities(eps, o, v, B_ov):
    """Gv, Ev, Go, Eo (as in dense.second_order_intermediates), each sum over the first
    occupied index k taken one k at a time: for fixed k the amplitudes t_kl^bd form an
    (o, v, v) array, so no o^2 v^2 array is held."""
    eo, ev = eps[:o], eps[o:]
    naux = B_ov.shape[0]
    L = B_ov.reshape(naux, o * v)
    Gv = np.zeros((v, v))
    Ev = np.zeros((v, v))
    Go = np.zeros((o, o))
    Eo = np.zeros((o, o))
    for k in range(o):
        kbld = (np.ascontiguousarray(L.reshape(naux, o, v)[:, k, :]).T @ L).reshape(v, o, v)             # (kb|ld) [b][l][d]
        D = eo[k] + eo[:, None, None] - ev[None, :, None] - ev[None, None, :]      # [l][b][d]
        t = np.transpose(kbld, (1, 0, 2)) / D                                      # t_kl^bd [l][b][d]
        tau = 2.0 * t - np.transpose(t, (0, 2, 1))                                 # tau_kl^bd
        # Gv_ab += sum_ld tau_kl^ad t_kl^bd ;  Ev with weight eps_k + eps_l - eps_d
        w = eo[k] + eo[:, None] - ev[None, :]                                      # [l][d]
        ta = np.transpose(tau, (1, 0, 2)).reshape(v, o * v)                        # [a][(l,d)]
        tb = np.transpose(t, (1, 0, 2)).reshape(v, o * v)
        Gv += ta @ tb.T
        Ev += ta @ (tb * w.reshape(1, o * v)).T
        # Go_ij += sum_cd tau_ik^cd t_jk^cd, with tau_ik^cd = tau_ki^dc, t_jk^cd = t_kj^dc;
        # Eo with weight eps_k - eps_c - eps_d (symmetric in c, d)
        wo = (eo[k] - ev[:, None] - ev[None, :]).reshape(1, v * v)
        ti = tau.reshape(o, v * v)
        tj = t.reshape(o, v * v)
        Go += ti @ tj.T
        Eo += ti @ (tj * wo).T
    return dict(Gv=Gv, Ev=Ev, Go=Go, Eo=Eo)


def second_order_rows(eps, o, v, B_oo, B_ov, B_vv, rows, V, dens=None):
    """(A V)[:, ia], (B V)[:, ia] and (S V)[:, ia] of the complete matrices through second
    order (orders 0 + 1 + 2) for the sampled compound indices 'rows'.

    V is (k, o*v).  dens: the MP2 densities (mp2_densities); without them only B is
    returned complete and A, S come back as None (their second-order rows need the
    densities, whose cost is that of the whole amplitude set).
    Returns (AV, BV, SV), each (k, len(rows)) or None.
    """
    eo, ev = eps[:o], eps[o:]
    naux = B_ov.shape[0]
    Boo_i = [B_oo[:, int(ia) // v, :] for ia in rows]
    Bvv_a = [B_vv[:, int(ia) % v, :] for ia in rows]
    AV1, BV1 = first_order_rows(eps, o, v, B_ov, rows, Boo_i, Bvv_a, V)
    k = V.shape[0]
    BV = BV1.copy()
    for t, ia in enumerate(rows):
        BV[:, t] += V @ b2_row(eps, o, v, B_oo, B_ov, B_vv, ia).reshape(o * v)
    if dens is None:
        return None, BV, None
    Gv, Ev, Go, Eo = dens["Gv"], dens["Ev"], dens["Go"], dens["Eo"]
    Vr = V.reshape(k, o, v)
    AV = AV1.copy()
    SV = np.zeros((k, len(rows)))
    for t, ia in enumerate(rows):
        i, a = divmod(int(ia), v)
        # rows of S2 and A2: -Go_ij V_ja - Gv_ab V_ib ; -(Ev_ab - eps_i Gv_ab) V_ib - (eps_a Go_ij + Eo_ij) V_ja
        SV[:, t] = V[:, ia] - Vr[:, :, a] @ Go[i] - Vr[:, i, :] @ Gv[a]
        AV[:, t] += -Vr[:, i, :] @ (Ev[a] - eo[i] * Gv[a]) - Vr[:, :, a] @ (ev[a] * Go[i] + Eo[i])
    return AV, BV, SV
