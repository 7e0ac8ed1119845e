"""Writes the stored expected values of the window-solve workloads.

Calls only the FP64 oracle (dense assembly and exact pencil diagonalisation) on
the seeded synthetic systems; no value comes from the HIP path.  Usage:
    python tests/golden/make_golden.py [workload ...]
Each workload produces tests/golden/<workload>.json with, per window, the
oracle's roots nearest omega0 (Ha, ascending) and their dipole oscillator
strengths.  Second-order workloads also get a "survey": 24 windows from 0.35 to
1.5 Ha (10 roots each, energies only) that exercise the completeness of the
window solver across the spectrum.  A serving request (one system of the serving
stream's shape, n_vir = 4 n_occ and n_aux = 12 n_occ, with one window) is written
the same way under its own name.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth.gen import CONFIGS, WINDOWS, gen, gen_config  # noqa: E402
from oracle import dense, pencil  # noqa: E402


def make(name):
    cfg = CONFIGS[name]
    omegas, nr = WINDOWS[name]
    t0 = time.time()
    sys_ = gen_config(name)
    A, B, S = dense.assemble(sys_, cfg["order"])
    om, X, Y = pencil.solve_all(A, B, S)
    out = dict(workload=name, order=cfg["order"], o=cfg["o"], v=cfg["v"], naux=cfg["naux"], seed=cfg["seed"],
               mp2_energy=dense.mp2_energy(sys_) if cfg["order"] >= 2 else 0.0, windows=[])
    for w0 in omegas:
        idx = pencil.select_window(om, float(w0), nr)
        idx = idx[np.argsort(om[idx])]
        f = pencil.oscillator_strengths(om[idx], X[:, idx], Y[:, idx], sys_.dip)
        out["windows"].append(dict(omega0=float(w0), n_roots=int(nr), energies=[float(x) for x in om[idx]],
                                   osc=[float(x) for x in f]))
    if cfg["order"] >= 2:
        out["survey"] = []
        for w0 in np.linspace(0.35, 1.5, 24):
            idx = pencil.select_window(om, float(w0), 10)
            out["survey"].append(dict(omega0=float(w0), n_roots=10, energies=[float(x) for x in np.sort(om[idx])]))
    out["oracle_seconds"] = time.time() - t0
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, f"({out['oracle_seconds']:.1f} s)")


# serving requests: name -> (seed, n_occ, omega0, n_roots); n_vir = 4 n_occ, n_aux = 12 n_occ
REQUESTS = {"serve_o40_v160_x480": (4040, 40, 0.8, 8)}


def make_request(name):
    seed, o, w0, nr = REQUESTS[name]
    t0 = time.time()
    sys_ = gen(seed, o, 4 * o, 12 * o)
    A, B, S = dense.assemble(sys_, 2)
    om, X, Y = pencil.solve_all(A, B, S)
    idx = pencil.select_window(om, float(w0), nr)
    idx = idx[np.argsort(om[idx])]
    f = pencil.oscillator_strengths(om[idx], X[:, idx], Y[:, idx], sys_.dip)
    out = dict(request=name, order=2, o=o, v=4 * o, naux=12 * o, seed=seed, omega0=float(w0), n_roots=int(nr),
               energies=[float(x) for x in om[idx]], osc=[float(x) for x in f],
               oracle_seconds=time.time() - t0)
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, f"({out['oracle_seconds']:.1f} s)")


if __name__ == "__main__":
    names = sys.argv[1:] or ["rpa1_o8_v24_x64", "mp2_o40_v160_x600"] + list(REQUESTS)
    for n in names:
        make_request(n) if n in REQUESTS else make(n)
