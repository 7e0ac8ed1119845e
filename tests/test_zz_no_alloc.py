"""pp_sigma_static, the product for callers that cannot allocate, through the C ABI:
the same result as pp_sigma on the same handle (same kernels and workspaces, staging in
the library's fixed scratch array instead of handle allocations), on two calls in a row
with the second smaller, with nothing allocated by either call."""
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


@pytest.mark.parametrize("precision", ["fp64", "sbf16"])
def test_sigma_static_matches_sigma(P, precision):
    import torch
    sys_ = gen(7, 12, 40, 100, b_scale=0.3)
    X1, X2 = random_block(21, sys_.N, 5), random_block(22, sys_.N, 2)
    reduced = precision == "sbf16"
    prec = P.PP_SPLIT_BF16 if reduced else P.PP_FP64
    print(f"[static] precision={precision}", flush=True)
    with P.Handle.from_system(sys_, order=2, store_amplitudes=0, strip_rows=3, precision=prec) as h:
        d1, d2 = torch.tensor(X1, device="cuda"), torch.tensor(X2, device="cuda")
        ref1, ref2 = torch.empty_like(d1), torch.empty_like(d2)
        h.sigma_device(d1, ref1, reduced=reduced)     # reserves the workspace for 5 vectors
        h.sigma_device(d2, ref2, reduced=reduced)
        refS = torch.empty_like(d2)
        h.sigma_device(d2, refS, metric=True, reduced=reduced)
        torch.cuda.synchronize()
        used = h.device_bytes()
        out1 = torch.full_like(d1, float("nan"))
        out2 = torch.full_like(d2, float("nan"))
        outS = torch.full_like(d2, float("nan"))
        h.sigma_static(d1, out1, reduced=reduced)
        h.sigma_static(d2, out2, reduced=reduced)     # second call, smaller input
        h.sigma_static(d2, outS, metric=True, reduced=reduced)
        torch.cuda.synchronize()
        assert h.device_bytes() == used
    assert torch.equal(out1, ref1) and torch.equal(out2, ref2) and torch.equal(outS, refS)
    if not reduced:
        for X, out in ((X1, out1), (X2, out2)):
            ref = dense.sigma_dense(sys_, 2, X)
            np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_sigma_static_refusals(P):
    """Refused with PP_EINVAL, before any work: a workspace not yet reserved for 2m vectors,
    staging beyond the fixed scratch (4 * 2m * N > 8 Mi doubles)."""
    import torch
    sys_ = gen(11, 5, 19, 23, b_scale=0.5)
    X = torch.tensor(random_block(3, sys_.N, 4), device="cuda")
    out = torch.empty_like(X)
    with P.Handle.from_system(sys_, order=2) as h:
        with pytest.raises(P.PPError) as e:
            h.sigma_static(X, out)
        assert e.value.status == P.PP_EINVAL
        m = (8 << 20) // (8 * sys_.N) + 1
        big = torch.zeros((m, 2, sys_.N), dtype=torch.float64, device="cuda")
        h.sigma_device(big[:1], torch.empty_like(big[:1]))
        with pytest.raises(P.PPError) as e:
            h.sigma_static(big, torch.empty_like(big))
        assert e.value.status == P.PP_EINVAL
