"""The C-ABI library loads without a GPU and exports every function the public headers declare.

No compute entry point is called here (there is no device); the host-only helpers
(pp_default_options, pp_status_string) are, since they touch no device state.
"""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_09811_amd", "libppwin.so")


def _declared():
    names = []
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        names += re.findall(r"\b((?:pp|ppint)_\w+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libppwin.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_headers_declare_the_boundary():
    names = _declared()
    for required in ("pp_setup", "pp_sigma", "pp_window_solve", "pp_window_solve_batch", "pp_destroy",
                     "pp_status_string", "pp_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_host_only_helpers(lib):
    import paper_2512_09811_amd.binding as b
    opt = b.pp_options()
    lib.pp_default_options(ctypes.byref(opt))
    assert opt.precision == 0 and opt.tol == 1e-9 and opt.max_cycles > 0
    lib.pp_status_string.restype = ctypes.c_char_p
    for code in range(7):
        assert lib.pp_status_string(code)


def test_spectrum_host_entry():
    """pp_spectrum (host-only): each root contributes a unit-area Lorentzian times its
    oscillator strength; the integral over a wide grid is the sum of strengths, an
    isolated peak has height f/(pi eta), and bad arguments are rejected."""
    import numpy as np
    import paper_2512_09811_amd as P
    e = np.array([0.5, 0.9, 0.905, 2.0])
    f = np.array([0.1, 0.02, 0.3, 0.05])
    eta = 2e-3
    w = np.linspace(-50.0, 60.0, 2_000_001)
    s = P.spectrum(e, f, w, eta)
    integral = np.sum(0.5 * (s[1:] + s[:-1]) * np.diff(w))
    tails = (f.sum() * 2 * eta / np.pi) * (1 / 50.0)  # the Lorentzian mass outside the grid, to first order
    assert abs(integral - f.sum()) < tails
    peak = P.spectrum(e, f, np.array([2.0]), eta)[0]
    assert abs(peak - f[3] / (np.pi * eta)) < 1e-3 * peak
    with pytest.raises(P.PPError, match="eta must be positive"):
        P.spectrum(e, f, w[:10], 0.0)
