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
        ijab = (Boo_i[t].T @ Bvv_a[t]).reshape(o * v)        # (ij|ab): [j][b]
        ibja = (B_ov[:, :, a].T @ B_ov[:, i, :]).reshape(o * v)  # (ib|ja): [j][b]
        a_row = 2.0 * iajb - ijab
        b_row = 2.0 * iajb - ibja
        a_row[ia] += eps[o + a] - eps[i]
        AV[:, t] = V @ a_row
        BV[:, t] = V @ b_row
    return AV, BV
