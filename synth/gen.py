"""Seeded generator for synthetic closed-shell systems.

The paper's systems are PbS and CdS quantum dots whose Hartree-Fock orbital
energies, density-fitted (DF) two-electron integrals and dipole integrals come
from an external electronic-structure code (Results section, the paragraph on
TeraChem and density fitting).  Those data are not available here, so this
module draws seeded stand-ins with the same shapes and with value
distributions chosen to mimic a gapped semiconductor:

* occupied energies  eps_i ~ sort(U[-1.0, -0.3]) Ha
* virtual energies   eps_a ~ sort(U[0.05, 2.0]) Ha
* DF factors         B_P = (0.05/sqrt(naux)) * (Z + Z^T)/2,  Z ~ N(0,1), n x n
  so that (pq|rs) = sum_P B_Ppq B_Prs is a positive semidefinite, 8-fold
  symmetric integral tensor (Results section, density fitting)
* dipole components  mu^x = (Z + Z^T)/2,  Z ~ 0.1 N(0,1)   (Discussion, the
  transition-strength paragraph)

The draw order is fixed: occupied energies, virtual energies, then one n x n
normal draw per auxiliary index P (orbitals ordered occupied first), then one
n x n draw per Cartesian dipole component.  Drawing B one P at a time keeps the
peak host memory at n^2 doubles beyond the output.

Only the oo, ov and vv blocks of B and the ov block of the dipoles are kept;
those are all a particle-hole response calculation reads.

The PCG64 generator of numpy (``numpy.random.default_rng(seed)``) is the single
source of randomness.  Nothing here contracts, divides or solves.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Workload sizes.  Keys name the workload by what it is.
CONFIGS = {
    # first-order (RPA A/B) window solve, FP64
    "rpa1_o8_v24_x64": dict(o=8, v=24, naux=64, order=1, seed=1),
    # second-order (MP2-corrected A/B) window solves, FP64, amplitudes stored
    "mp2_o40_v160_x600": dict(o=40, v=160, naux=600, order=2, seed=2),
    # PbS-dot-shaped second-order system, amplitudes built in strips
    "mp2_o200_v800_x3000": dict(o=200, v=800, naux=3000, order=2, seed=3),
    # largest matrix-free second-order system
    "mp2_o256_v1024_x4096": dict(o=256, v=1024, naux=4096, order=2, seed=5),
}

# Frequency windows (Hartree) and roots per window for each workload.
WINDOWS = {
    "rpa1_o8_v24_x64": (np.array([0.5]), 6),
    "mp2_o40_v160_x600": (np.array([0.3, 0.6, 0.9, 1.2]), 10),
    "mp2_o200_v800_x3000": (np.linspace(0.3, 1.2, 16), 8),
    "mp2_o256_v1024_x4096": (np.linspace(0.3, 1.2, 8), 16),
}

# Serving stream: request r is drawn from seed REQUEST_SEED_BASE + r.
REQUEST_SEED_BASE = 4000


@dataclasses.dataclass
class System:
    """One closed-shell system in the layout the C ABI takes.

    eps   : (o+v,)         occupied energies first, each block ascending
    B_oo  : (naux, o, o)   DF factors, occupied-occupied block
    B_ov  : (naux, o, v)   DF factors, occupied-virtual block
    B_vv  : (naux, v, v)   DF factors, virtual-virtual block
    dip   : (3, o, v)      dipole integrals, occupied-virtual block
    """

    o: int
    v: int
    naux: int
    eps: np.ndarray
    B_oo: np.ndarray
    B_ov: np.ndarray
    B_vv: np.ndarray
    dip: np.ndarray
    seed: Optional[int] = None

    @property
    def N(self) -> int:
        return self.o * self.v

    @property
    def eps_o(self) -> np.ndarray:
        return self.eps[: self.o]

    @property
    def eps_v(self) -> np.ndarray:
        return self.eps[self.o:]

    def scaled(self, s: float) -> "System":
        """Same system with every DF factor multiplied by s (integrals by s^2)."""
        return dataclasses.replace(self, B_oo=self.B_oo * s, B_ov=self.B_ov * s, B_vv=self.B_vv * s)


def gen(seed: int, o: int, v: int, naux: int, *, eps_occ=(-1.0, -0.3), eps_vir=(0.05, 2.0),
        b_scale: float = 0.05, dip_scale: float = 0.1) -> System:
    """Draw one synthetic system (see the module docstring for the recipe)."""
    if o < 1 or v < 1 or naux < 1:
        raise ValueError("o, v and naux must be positive")
    rng = np.random.default_rng(seed)
    e_o = np.sort(rng.uniform(eps_occ[0], eps_occ[1], o))
    e_v = np.sort(rng.uniform(eps_vir[0], eps_vir[1], v))
    n = o + v
    B_oo = np.empty((naux, o, o))
    B_ov = np.empty((naux, o, v))
    B_vv = np.empty((naux, v, v))
    pref = b_scale / np.sqrt(naux)
    for P in range(naux):
        Z = rng.standard_normal((n, n))
        S = pref * 0.5 * (Z + Z.T)
        B_oo[P] = S[:o, :o]
        B_ov[P] = S[:o, o:]
        B_vv[P] = S[o:, o:]
    dip = np.empty((3, o, v))
    for x in range(3):
        Z = dip_scale * rng.standard_normal((n, n))
        dip[x] = (0.5 * (Z + Z.T))[:o, o:]
    return System(o=o, v=v, naux=naux, eps=np.concatenate([e_o, e_v]), B_oo=B_oo, B_ov=B_ov,
                  B_vv=B_vv, dip=dip, seed=seed)


def gen_config(name: str) -> System:
    c = CONFIGS[name]
    return gen(c["seed"], c["o"], c["v"], c["naux"])


def gen_request(r: int, o_min: int = 16, o_max: int = 128):
    """Serving-stream request r: its system and (omega0, n_roots).

    n_occ ~ U{o_min..o_max} (16..128 for the full stream), n_vir = 4 n_occ,
    n_aux = 12 n_occ, omega0 ~ U[0.3, 1.5], n_roots ~ U{4..12}; the request
    parameters are drawn first from the same seeded stream as the system.
    """
    rng = np.random.default_rng(REQUEST_SEED_BASE + r)
    o = int(rng.integers(o_min, o_max + 1))
    omega = float(rng.uniform(0.3, 1.5))
    nroots = int(rng.integers(4, 13))
    sys_seed = int(rng.integers(0, 2**31 - 1))
    return gen(sys_seed, o, 4 * o, 12 * o), omega, nroots


def random_block(seed: int, N: int, m: int) -> np.ndarray:
    """Seeded trial-vector block [m][2][N] (rows are [X;Y] pairs), N(0,1) entries."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, 2, N))
