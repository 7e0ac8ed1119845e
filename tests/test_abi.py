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
    # last field of the struct: the binding's layout matches the header's
    assert opt.contour_maxit == 500 and opt.pass_vectors == 0
    lib.pp_status_string.restype = ctypes.c_char_p
    for code in range(7):
        assert lib.pp_status_string(code)


def test_spectrum_and_response_argument_checks():
    """pp_spectrum and pp_response refuse bad arguments before any device work."""
    import numpy as np
    import paper_2512_09811_amd as P
    e = np.array([0.5, 0.9])
    f = np.array([0.1, 0.02])
    w = np.linspace(0.0, 1.0, 10)
    with pytest.raises(P.PPError, match="eta must be positive"):
        P.spectrum(e, f, w, 0.0)
    with pytest.raises(P.PPError, match="eta must be >= 0"):
        P.response(e, f, w, -1e-3)
    with pytest.raises(P.PPError, match="energies must be positive"):
        P.response(np.array([0.5, -0.1]), f, w, 1e-3)
    with pytest.raises(P.PPError, match="energies must be positive"):
        P.spectrum(np.array([0.5, np.nan]), f, w, 1e-3)
