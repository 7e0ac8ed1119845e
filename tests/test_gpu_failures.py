"""Failure paths forced from the host, through the C ABI: an unstable response matrix
(A - B indefinite), a diagonal of the shifted pencil that vanishes at omega0 (clamped),
and HIP errors injected in place of a runtime call's return value.  No kernel is made to
fault: every launch runs normally."""
import numpy as np
import pytest

from synth import gen
from oracle import dense, pencil

pytestmark = pytest.mark.gpu

HIP_ERROR_LAUNCH_FAILURE = 719


@pytest.fixture(scope="module")
def P():
    import paper_2512_09811_amd as P
    P.lib()
    return P


def test_unstable_response_matrix(P):
    """Integrals scaled by 10: A - B is indefinite (even on its diagonal), which the real
    roots of the generalized eigenvalue equation exclude; the oracle refuses the system and
    the library's window solve returns PP_EUNSTABLE with its message."""
    sys_ = gen(11, 5, 19, 23, b_scale=10.0)
    A, B, S = dense.assemble(sys_, 1)
    assert np.linalg.eigvalsh(A - B).min() < 0
    with pytest.raises(pencil.NotStable):
        pencil.solve_all(A, B, S)
    with P.Handle.from_system(sys_, order=1) as h:
        with pytest.raises(P.PPError) as e:
            h.window_solve(0.8, 4)
        assert e.value.status == P.PP_EUNSTABLE
        assert "positive definite" in str(e.value)


@pytest.mark.parametrize("order", [1, 2])
def test_clamped_diagonal_at_omega0(P, order):
    """omega0 placed exactly on a diagonal element of A (the Jacobi splitting's D vanishes
    there and is clamped to d_clamp): the converged roots are the oracle's, unchanged by
    the clamp, and the same as those of a window shifted by 1e-3 Ha where they overlap."""
    sys_ = gen(7, 12, 40, 100, b_scale=0.3)
    A, B, S = dense.assemble(sys_, order)
    dA = np.diag(A)
    ia = int(np.argsort(dA)[len(dA) // 3])
    omega0 = float(dA[ia] / S[ia, ia])
    e_ref, _, _, f_ref = pencil.window_solve(A, B, S, sys_.dip, omega0, 6)
    with P.Handle.from_system(sys_, order=order) as h:
        e, _, f, info = h.window_solve(omega0, 6)
        e2, _, _, _ = h.window_solve(omega0 + 1e-3, 6)
    assert np.all(info["converged"] == 1)
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-8)
    big = f_ref >= 1e-4 * f_ref.max()
    np.testing.assert_allclose(f[big], f_ref[big], rtol=1e-5)
    common = [x for x in e if np.min(np.abs(e2 - x)) < 1e-6]
    assert len(common) >= 4
    for x in common:
        assert np.min(np.abs(e2 - x)) < 1e-8


def test_injected_hip_errors(P):
    """A HIP error reported in place of a runtime call's return value: during setup the
    setup fails with PP_EDEVICE (no handle) and the error's message; during a window solve
    the solve fails with PP_EDEVICE; afterwards the same handle solves the window again
    and matches the oracle, and a fresh handle works too."""
    sys_ = gen(11, 5, 19, 23, b_scale=0.5)
    A, B, S = dense.assemble(sys_, 2)
    e_ref, _, _, _ = pencil.window_solve(A, B, S, sys_.dip, 0.9, 4)
    P.inject_hip_error(1, HIP_ERROR_LAUNCH_FAILURE)
    with pytest.raises(P.PPError) as e:
        P.Handle.from_system(sys_, order=2)
    P.inject_hip_error(0)
    assert e.value.status == P.PP_EDEVICE
    with P.Handle.from_system(sys_, order=2) as h:
        for after in (5, 60, 400):
            P.inject_hip_error(after, HIP_ERROR_LAUNCH_FAILURE)
            with pytest.raises(P.PPError) as e:
                h.window_solve(0.9, 4)
            P.inject_hip_error(0)
            assert e.value.status == P.PP_EDEVICE, after
            got, _, _, info = h.window_solve(0.9, 4)
            np.testing.assert_allclose(got, e_ref, rtol=0, atol=1e-8)
    with pytest.raises(P.PPError):
        P.inject_hip_error(-1, HIP_ERROR_LAUNCH_FAILURE)
    with P.Handle.from_system(sys_, order=2) as h:
        got, _, _, _ = h.window_solve(0.9, 4)
    np.testing.assert_allclose(got, e_ref, rtol=0, atol=1e-8)
