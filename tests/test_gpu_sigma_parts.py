"""Products issued in parts (pp_sigma_part) and in the handle's reduced precision
(PP_REDUCED), through the C ABI, against the dense FP64 oracle and against the
same product issued in one call."""
import numpy as np
import pytest

from synth import gen
from synth.gen import random_block
from oracle import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2512_09811_amd as P
    P.lib()
    return P


@pytest.mark.parametrize("n_parts", [1, 4, 5, 12])
def test_sigma_parts_match_oracle(P, n_parts):
    """Second-order products in n_parts calls (amplitudes rebuilt in strips of 3 occupied
    rows; 5 parts cut strips differently) match the oracle element by element at 1e-12
    of the largest element, and the one-call product at the same bar; host and device
    pointers, with and without the metric."""
    import torch
    sys = gen(7, 12, 40, 100, b_scale=0.3)
    print(f"[parts] n_parts={n_parts}", flush=True)
    X = random_block(3, sys.N, 4)
    ref = dense.sigma_dense(sys, 2, X)
    refS = dense.sigma_dense(sys, 2, X, metric=True)
    with P.Handle.from_system(sys, order=2, store_amplitudes=0, strip_rows=3) as h:
        one = h.sigma(X)
        out = np.empty_like(X)
        for p in range(n_parts):
            h.sigma_part(X, out, p, n_parts)
        dX = torch.tensor(X, device="cuda")
        dout = torch.empty_like(dX)
        for p in range(n_parts):
            h.sigma_part(dX, dout, p, n_parts, metric=True)
        outS = dout.cpu().numpy()
    scale = np.abs(ref).max()
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(out, one, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(outS, refS, rtol=0, atol=1e-13)
    if n_parts == 4:
        # parts that follow the strips exactly: bit-identical to the one-call product
        assert np.array_equal(out, one)


@pytest.mark.parametrize("precision", ["fp32", "sbf16"])
def test_sigma_reduced_parts(P, precision):
    """PP_REDUCED products (FP32 contractions, the amplitude ones split-BF16 in sbf16
    mode) in one call and in parts agree with each other to rounding and with the oracle
    to the reduced precision on the second-order part; PP_REDUCED on an FP64 handle is
    refused with PP_ENOTSUP."""
    sys = gen(11, 5, 19, 23, b_scale=0.5)
    X = random_block(8, sys.N, 3)
    ref = dense.sigma_dense(sys, 2, X)
    ref1 = dense.sigma_dense(sys, 1, X)
    prec = P.PP_FP32 if precision == "fp32" else P.PP_SPLIT_BF16
    with P.Handle.from_system(sys, order=2, store_amplitudes=0, strip_rows=2, precision=prec) as h:
        one = h.sigma(X, reduced=True)
        out = np.empty_like(X)
        for p in range(3):
            h.sigma_part(X, out, p, 3, reduced=True)
    second = np.abs(ref - ref1).max()
    assert np.abs(one - ref).max() <= 1e-4 * second + 1e-12
    assert np.abs(out - ref).max() <= 1e-4 * second + 1e-12
    assert np.abs(out - one).max() <= 1e-5 * second + 1e-13
    with P.Handle.from_system(sys, order=2) as h:
        with pytest.raises(P.PPError) as e:
            h.sigma(X, reduced=True)
        assert e.value.status == P.PP_ENOTSUP


def test_sigma_parts_errors(P):
    """Parts out of order, with other arguments, after another product on the handle, or
    with n_parts outside 1..n_occ are refused with PP_EINVAL; a refused sequence can be
    started again at part 0 and then completes correctly."""
    sys = gen(11, 5, 19, 23, b_scale=0.5)
    X = random_block(9, sys.N, 2)
    ref = dense.sigma_dense(sys, 2, X)
    out = np.empty_like(X)
    with P.Handle.from_system(sys, order=2, store_amplitudes=0, strip_rows=2) as h:
        for bad in (0, 6):
            with pytest.raises(P.PPError) as e:
                h.sigma_part(X, out, 0, bad)
            assert e.value.status == P.PP_EINVAL
        with pytest.raises(P.PPError) as e:
            h.sigma_part(X, out, 1, 3)          # no pass in progress
        assert e.value.status == P.PP_EINVAL
        h.sigma_part(X, out, 0, 3)
        with pytest.raises(P.PPError) as e:
            h.sigma_part(X, out, 2, 3)          # skips part 1
        assert e.value.status == P.PP_EINVAL
        with pytest.raises(P.PPError) as e:
            h.sigma_part(X, out, 1, 4)          # other n_parts
        assert e.value.status == P.PP_EINVAL
        h.sigma(X)                              # another product in between
        with pytest.raises(P.PPError) as e:
            h.sigma_part(X, out, 1, 3)
        assert e.value.status == P.PP_EINVAL
        for p in range(3):
            h.sigma_part(X, out, p, 3)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
