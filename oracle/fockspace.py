"""Brute-force Fock-space evaluation of the defining expectation values.

Test infrastructure (see the package docstring): never used by the product.

Everything is an explicit matrix over the Slater determinants of a fixed
particle number: H is built from one- and two-electron integrals, the
normal-ordered pieces H0 = sum_p eps_p {p^+ p} and W_N = H_N - H0 follow from
H_N = H - <0|H|0> (Theory section, MP2 paragraph), and the MP2 first-order
wavefunction is R0 W_N |0> with R0 the zeroth-order resolvent.  The response
elements are then the expectation values the paper defines, evaluated by
applying the ph operators q_ai = i^+ a and q^+_ai = a^+ i to state vectors:

* metric     S_{ai,bj} = <[q_ai, q^+_bj]>
* A block    symmetrized double commutator 1/2 <[q,[H,q^+]] + [[q,H],q^+]>
* B block    -<[q_ai, [H, q_bj]]> (sign chosen so that B1 = <ab||ij>)

with <.> over the normalized |0> + Psi1, kept to second order in W_N:
order-2 part of <O> = <Psi1|O|Psi1> - <Psi1|Psi1><0|O|0> + <Psi1|O_W|0> + <0|O_W|Psi1>,
where O_W is the W_N part of O.  This is the second-order expansion of the
superoperator matrix element over the MP2 ground state (reading R2: the
W-cross terms enter A as they enter B).  Small systems only (a few hundred
determinants).
"""
from __future__ import annotations

import itertools

import numpy as np


class FockSpace:
    """Determinants of n_el fermions in n_so orbitals; |0> = lowest n_el occupied."""

    def __init__(self, n_so: int, n_el: int):
        self.n_so, self.n_el = n_so, n_el
        self.dets = [sum(1 << p for p in occ) for occ in itertools.combinations(range(n_so), n_el)]
        self.index = {d: k for k, d in enumerate(self.dets)}
        self.dim = len(self.dets)
        self.ref = self.index[(1 << n_el) - 1]

    @staticmethod
    def _apply(det, p, create):
        """a_p^+ (create) or a_p on a bit-string determinant -> (sign, det) or None."""
        occ = (det >> p) & 1
        if create == bool(occ):
            return None
        sign = -1 if bin(det & ((1 << p) - 1)).count("1") % 2 else 1
        return sign, det ^ (1 << p)

    def excitation_matrix(self, p, q):
        """Matrix of p^+ q (particle-number conserving) in this sector."""
        M = np.zeros((self.dim, self.dim))
        for k, d in enumerate(self.dets):
            r1 = self._apply(d, q, False)
            if r1 is None:
                continue
            r2 = self._apply(r1[1], p, True)
            if r2 is None:
                continue
            M[self.index[r2[1]], k] += r1[0] * r2[0]
        return M

    def hamiltonian(self, eps, V):
        """H with Fock matrix diag(eps) w.r.t. |0>, two-electron part 1/4 <pq||rs> p^+ q^+ s r.

        h_pq = eps_p delta_pq - sum_i <pi||qi> makes the Fock operator diagonal,
        so that H_N = sum eps_p {p^+ p} + W_N exactly.
        Returns (H, E) with E[p, q] the matrices of p^+ q.
        """
        n, no = self.n_so, self.n_el
        E = np.array([[self.excitation_matrix(p, q) for q in range(n)] for p in range(n)])
        h = np.diag(eps) - np.einsum("piqi->pq", V[:, :no, :, :no])
        H1 = np.einsum("pq,pqxy->xy", h, E)
        # p^+ q^+ s r = E_pr E_qs - delta_qr E_ps
        T = np.tensordot(V, E, axes=([1, 3], [0, 1]))          # [p, r, x, y] = sum_qs V_pqrs E_qs
        H2 = np.einsum("prxy,pryz->xz", E, T)
        H2 -= np.einsum("pqqs,psxy->xy", V, E)
        return H1 + 0.25 * H2, E


class MP2Response:
    """Second-order S, A, B of the MP2 ground state by direct evaluation."""

    def __init__(self, eps, n_occ, V):
        n = len(eps)
        self.no, self.nv = n_occ, n - n_occ
        fs = FockSpace(n, n_occ)
        self.fs = fs
        H, E = fs.hamiltonian(eps, V)
        ref = np.zeros(fs.dim)
        ref[fs.ref] = 1.0
        e_hf = ref @ H @ ref
        HN = H - e_hf * np.eye(fs.dim)
        occ_sum = float(np.sum(eps[:n_occ]))
        H0 = np.einsum("p,ppxy->xy", eps, E) - occ_sum * np.eye(fs.dim)
        W = HN - H0
        self.H0, self.W, self.ref = H0, W, ref
        e0 = np.diag(H0)
        w0 = W @ ref
        psi1 = np.zeros(fs.dim)
        mask = np.arange(fs.dim) != fs.ref
        psi1[mask] = w0[mask] / (e0[fs.ref] - e0[mask])
        self.psi1 = psi1
        self.E = E
        # ph operators: exc[k] = a^+ i, dex[k] = i^+ a, k = i*nv + a
        no, nv = self.no, self.nv
        self.exc = np.array([E[no + a, i] for i in range(no) for a in range(nv)])
        self.dex = np.array([E[i, no + a] for i in range(no) for a in range(nv)])

    # --- scalar pieces -------------------------------------------------------
    def mp2_energy(self):
        return float(self.ref @ self.W @ self.psi1)

    def brillouin_max(self):
        """max |<S|H_N|0>| over singly excited S (zero for a diagonal Fock operator)."""
        singles = self.exc @ self.ref
        return float(np.max(np.abs(singles @ (self.H0 + self.W) @ self.ref)))

    # --- generic commutator expectation values ------------------------------
    def _dc(self, L, O, R, Qs, Qps):
        """<L|[Q_k,[O,Qp_l]]|R> for all k, l (Qs: list of Q, Qps: list of Qp)."""
        # [Q,[O,Qp]] = Q O Qp - Q Qp O - O Qp Q + Qp O Q
        QtL = np.einsum("kxy,x->ky", Qs, L)          # (Q^T L)  -> <L|Q = (Q^T L)^T
        QpR = np.einsum("lxy,y->lx", Qps, R)
        QpOR = np.einsum("lxy,y->lx", Qps, O @ R)
        OtL = O.T @ L
        QR = np.einsum("kxy,y->kx", Qs, R)
        QptL = np.einsum("lxy,x->ly", Qps, L)
        QpQR = np.einsum("lxy,ky->klx", Qps, QR)
        t1 = QtL @ O @ QpR.T
        t2 = QtL @ QpOR.T
        t3 = np.einsum("x,klx->kl", OtL, QpQR)
        t4 = (QptL @ O @ QR.T).T
        return t1 - t2 - t3 + t4

    def _dc_other(self, L, O, R, Qs, Qps):
        """<L|[[Q_k,O],Qp_l]|R> = <L| Q O Qp - O Q Qp - Qp Q O + Qp O Q |R>."""
        QtL = np.einsum("kxy,x->ky", Qs, L)
        QpR = np.einsum("lxy,y->lx", Qps, R)
        OtL = O.T @ L
        QQpR = np.einsum("kxy,ly->klx", Qs, QpR)
        QptL = np.einsum("lxy,x->ly", Qps, L)
        QOR = np.einsum("kxy,y->kx", Qs, O @ R)
        QR = np.einsum("kxy,y->kx", Qs, R)
        t1 = QtL @ O @ QpR.T
        t2 = np.einsum("x,klx->kl", OtL, QQpR)
        t3 = (QptL @ QOR.T).T
        t4 = (QptL @ O @ QR.T).T
        return t1 - t2 - t3 + t4

    def _comm(self, L, R, Qs, Qps):
        """<L|[Q_k, Qp_l]|R>."""
        QtL = np.einsum("kxy,x->ky", Qs, L)
        QpR = np.einsum("lxy,y->lx", Qps, R)
        QptL = np.einsum("lxy,x->ly", Qps, L)
        QR = np.einsum("kxy,y->kx", Qs, R)
        return QtL @ QpR.T - (QptL @ QR.T).T

    def property_vector(self, d):
        """(F0, F2): F_k = <[Q_k, D]> for the one-body operator D = sum_pq d_pq p^+ q
        (the property vector of the propagator's numerator, Theory section), over the
        normalized |0> + Psi1 to second order.  The first-order terms <0|[Q,D]|Psi1> + c.c.
        are kept (they vanish: [Q, D] is one-body and Psi1 has only doubles)."""
        r, p = self.ref, self.psi1
        D = np.einsum("pq,pqxy->xy", d, self.E)
        C = np.einsum("kxy,yz->kxz", self.dex, D) - np.einsum("xy,kyz->kxz", D, self.dex)
        F0 = np.einsum("x,kxy,y->k", r, C, r)
        F1 = np.einsum("x,kxy,y->k", p, C, r) + np.einsum("x,kxy,y->k", r, C, p)
        F2 = np.einsum("x,kxy,y->k", p, C, p) - (p @ p) * F0
        return F0, F1 + F2

    # --- matrices by order ---------------------------------------------------
    def metric(self):
        """(S0, S2)."""
        r, p = self.ref, self.psi1
        S0 = self._comm(r, r, self.dex, self.exc)
        S2 = self._comm(p, p, self.dex, self.exc) - (p @ p) * S0
        return S0, S2

    def a_block(self):
        """(A0, A1, A2) with the symmetrized double commutator."""
        r, p = self.ref, self.psi1
        Q, Qp = self.dex, self.exc

        def sym(L, O, R):
            return 0.5 * (self._dc(L, O, R, Q, Qp) + self._dc_other(L, O, R, Q, Qp))

        A0 = sym(r, self.H0, r)
        A1 = sym(r, self.W, r)
        A2 = sym(p, self.H0, p) - (p @ p) * A0 + sym(p, self.W, r) + sym(r, self.W, p)
        return A0, A1, A2

    def a2_parts(self):
        """Second-order A split into the H0 (literal reading) and W-cross parts."""
        r, p = self.ref, self.psi1
        Q, Qp = self.dex, self.exc

        def sym(L, O, R):
            return 0.5 * (self._dc(L, O, R, Q, Qp) + self._dc_other(L, O, R, Q, Qp))

        h0_part = sym(p, self.H0, p) - (p @ p) * sym(r, self.H0, r)
        w_part = sym(p, self.W, r) + sym(r, self.W, p)
        return h0_part, w_part

    def b_block(self):
        """(B1, B2); B0 = 0.  Sign: B = -<[q_ai,[H,q_bj]]>."""
        r, p = self.ref, self.psi1
        Q = self.dex
        B0 = -self._dc(r, self.H0, r, Q, Q)
        B1 = -self._dc(r, self.W, r, Q, Q)
        B2 = -(self._dc(p, self.H0, p, Q, Q) - (p @ p) * (-B0)
               + self._dc(p, self.W, r, Q, Q) + self._dc(r, self.W, p, Q, Q))
        return B0, B1, B2
