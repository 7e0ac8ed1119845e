"""Spin-orbital route: A, B, S in a general (real) spin-orbital basis.

Test infrastructure (see the package docstring): never used by the product.

Model (Theory section, MP2 paragraph): H_N = sum_p eps_p {p^+ p} + W_N with
W_N = 1/4 sum <pq||rs> {p^+ q^+ s r}; the first-order wavefunction is
R0 W_N |0> = 1/4 sum t_ij^ab a^+ b^+ j i |0> with t_ij^ab = <ab||ij> / D_ij^ab.

The closed forms below are the second-order expansion of the defining
expectation values (metric <[q, q^+]>, symmetrized double commutator for A,
double commutator for B) over |0> + R0 W_N |0>.  The paper prints the defining
expectation values, not these closed forms, so they are pinned against the
brute-force evaluator in oracle.fockspace.

Basis of ph operators: q^+_{ai} = a^+ i, compound index ia = i*nv + a.
"""
from __future__ import annotations

import numpy as np


def antisym_from_chemist(eri):
    """<pq||rs> = (pr|qs) - (ps|qr) for a real chemists' tensor eri[p,q,r,s] = (pq|rs)."""
    phys = np.transpose(eri, (0, 2, 1, 3))          # <pq|rs> = (pr|qs)
    return phys - np.transpose(phys, (0, 1, 3, 2))


def spinorbital_system(sys):
    """Spin-orbital energies and <pq||rs> for a closed-shell spatial system.

    Spin orbitals are ordered occupied first; spatial orbital p gives spin
    orbitals 2p (alpha) and 2p+1 (beta) within its block.
    Returns (eps_so, n_occ_so, V) with V[p,q,r,s] = <pq||rs>.
    """
    o, v = sys.o, sys.v
    n = o + v
    B = np.zeros((sys.naux, n, n))
    B[:, :o, :o] = sys.B_oo
    B[:, :o, o:] = sys.B_ov
    B[:, o:, :o] = np.transpose(sys.B_ov, (0, 2, 1))
    B[:, o:, o:] = sys.B_vv
    eri = np.einsum("Ppq,Prs->pqrs", B, B)
    ns = 2 * n
    spat = np.arange(ns) // 2
    spin = np.arange(ns) % 2
    # spatial (pq|rs) with spin deltas delta(s_p, s_q) delta(s_r, s_s)
    eri_so = eri[np.ix_(spat, spat, spat, spat)]
    same_pq = (spin[:, None] == spin[None, :])
    mask = same_pq[:, :, None, None] & same_pq[None, None, :, :]
    eri_so = eri_so * mask
    V = antisym_from_chemist(eri_so)
    eps_so = np.repeat(sys.eps, 2)
    return eps_so, 2 * o, V


def spinless_system(seed, n_occ, n_vir, naux=6, scale=0.3):
    """A random real 'spinless' model: n_occ + n_vir orbitals, one fermion per orbital.

    (pq|rs) = sum_P B_Ppq B_Prs with symmetric random B_P; <pq||rs> is its
    antisymmetrized physicist form.  Used to exercise the spin-orbital closed
    forms with no spin structure that could hide a wrong term.
    """
    rng = np.random.default_rng(seed)
    n = n_occ + n_vir
    eps = np.concatenate([np.sort(rng.uniform(-1.2, -0.4, n_occ)), np.sort(rng.uniform(0.2, 1.6, n_vir))])
    Z = rng.standard_normal((naux, n, n))
    B = scale * 0.5 * (Z + np.transpose(Z, (0, 2, 1))) / np.sqrt(naux)
    eri = np.einsum("Ppq,Prs->pqrs", B, B)
    return eps, n_occ, antisym_from_chemist(eri)


def amplitudes(eps, no, V):
    """t[i,j,a,b] = <ab||ij> / (eps_i + eps_j - eps_a - eps_b)."""
    eo, ev = eps[:no], eps[no:]
    vvoo = V[no:, no:, :no, :no]                             # <ab||ij> [a,b,i,j]
    D = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return np.transpose(vvoo, (2, 3, 0, 1)) / D


def mp2_energy(eps, no, V):
    """1/4 sum_ijab t_ij^ab <ij||ab> (textbook spin-orbital MP2)."""
    t = amplitudes(eps, no, V)
    return 0.25 * float(np.einsum("ijab,ijab->", t, V[:no, :no, no:, no:]))


def assemble(eps, no, V, order: int):
    """Spin-orbital (A, B, S), index ia = i*nv + a; B sign: B1 = <ab||ij>."""
    ns = len(eps)
    nv = ns - no
    N = no * nv
    eo, ev = eps[:no], eps[no:]
    dI, dA = np.eye(no), np.eye(nv)
    A = np.diag((ev[None, :] - eo[:, None]).reshape(N))
    B = np.zeros((N, N))
    S = np.eye(N)
    if order == 0:
        return A, B, S
    o_, v_ = slice(0, no), slice(no, ns)
    # A1_{ia,jb} = <aj||ib>, B1_{ia,jb} = <ab||ij>
    A = A + np.einsum("ajib->iajb", V[v_, o_, o_, v_]).reshape(N, N)
    B = B + np.einsum("abij->iajb", V[v_, v_, o_, o_]).reshape(N, N)
    if order == 1:
        return A, B, S
    t = amplitudes(eps, no, V)
    # one-particle MP2 density pieces
    occ_dep = np.einsum("ikcd,jkcd->ij", t, t)               # sum_kcd t_ik^cd t_jk^cd
    vir_occ = np.einsum("klac,klbc->ab", t, t)               # sum_klc t_kl^ac t_kl^bc
    S2 = -0.5 * np.einsum("ab,ij->iajb", dA, occ_dep) - 0.5 * np.einsum("ij,ab->iajb", dI, vir_occ)
    # A2: delta-type terms only
    wv = eo[:, None, None] + eo[None, :, None] - ev[None, None, :]          # eps_k + eps_l - eps_d
    Tv = np.einsum("klad,klbd,kld->ab", t, t, wv)
    A2 = -0.5 * np.einsum("ij,ab->iajb", dI, Tv) + 0.5 * np.einsum("ij,i,ab->iajb", dI, eo, vir_occ)
    wo = eo[:, None, None] - ev[None, :, None] - ev[None, None, :]          # eps_k - eps_c - eps_d
    To = np.einsum("ikcd,jkcd,kcd->ij", t, t, wo)
    A2 += -0.5 * np.einsum("ab,ij->iajb", dA, To) - 0.5 * np.einsum("ab,a,ij->iajb", dA, ev, occ_dep)
    # B2
    B2 = (0.5 * np.einsum("abcd,ijcd->iajb", V[v_, v_, v_, v_], t)
          + 0.5 * np.einsum("klij,klab->iajb", V[o_, o_, o_, o_], t)
          - np.einsum("kbci,jkac->iajb", V[o_, v_, v_, o_], t)
          - np.einsum("kacj,ikbc->iajb", V[o_, v_, v_, o_], t))
    return A + A2.reshape(N, N), B + B2.reshape(N, N), S + S2.reshape(N, N)


def singlet_triplet_projection(Mso, o, v):
    """Project a spin-orbital ph matrix (closed-shell ordering) onto singlets and triplets.

    Spin-orbital ph pair (i sigma -> a sigma) of spatial pair (i, a); the singlet
    combination is (|a_alpha i_alpha> + |a_beta i_beta>)/sqrt(2), the (M_s = 0)
    triplet the difference.  Returns (singlet, triplet), each [o*v, o*v].
    """
    nv_so = 2 * v
    idx = np.zeros((2, o, v), dtype=int)
    for s in range(2):
        for i in range(o):
            for a in range(v):
                idx[s, i, a] = (2 * i + s) * nv_so + (2 * a + s)
    al = idx[0].reshape(-1)
    be = idx[1].reshape(-1)
    aa = Mso[np.ix_(al, al)]
    ab = Mso[np.ix_(al, be)]
    return aa + ab, aa - ab
