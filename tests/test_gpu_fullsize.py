"""Products at sizes where no dense oracle fits, through the C ABI, against the row
oracle (oracle.columns: single rows of the complete matrices from their element
form, pinned against the dense assembly at small sizes).

  * 96/384/1152 (particle-hole dimension 36,864; amplitudes rebuilt in strips of 7
    occupied rows, and stored): sampled rows of the complete A V, B V, S V through
    second order, element by element, to 1e-12 of the row scale, and their
    second-order parts to 1e-9 of their own scale;
  * 200/800/3000 (1.6e5) and 256/1024/4096 (2.6e5): sampled rows of the first-order
    A V, B V and, three and two of them, of the complete second-order B V (the
    amplitude-weighted ladder and ring terms; the A and S rows need the MP2 densities,
    the cost of the whole amplitude set on the host);
  * at both large sizes the projected matrices U^T (A U), U^T (B U), U^T (S U) of the
    second-order products are symmetric to rounding, and the metric is below the
    identity (occupation numbers of the MP2 state);
  * FP32 contractions agree with the FP64 path to single precision (smaller size).
Inputs of the two largest systems come from the seeded device generator (same recipe
as the numpy one); the 96/384/1152 system from the numpy generator.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

# (seed, o, v, naux, complete second-order B rows checked against the row oracle; about
# 25 s of host time each at the largest size)
CASES = {"mp2_o200_v800_x3000": (3, 200, 800, 3000, 3), "mp2_o256_v1024_x4096": (5, 256, 1024, 4096, 2)}


@pytest.fixture(scope="module")
def P():
    import paper_2512_09811_amd as P
    P.lib()
    return P


@pytest.mark.parametrize("name", list(CASES))
def test_fullsize_products(P, name):
    from synth.device_gen import gen_device
    from oracle import columns
    seed, o, v, X, b2_rows = CASES[name]
    N = o * v
    t0 = time.time()
    t = gen_device(seed, o, v, X)
    torch.cuda.synchronize()
    print(f"[fullsize] {name}: inputs drawn in {time.time() - t0:.1f} s", flush=True)
    k = 3 if b2_rows else 2
    rng = np.random.default_rng(seed + 100)
    U = torch.tensor(rng.standard_normal((k, N)), device="cuda")
    out = {key: torch.empty_like(U) for key in ("A1", "B1", "S1", "A2", "B2", "S2")}
    t0 = time.time()
    with P.Handle(t["eps"], t["B_oo"], t["B_ov"], t["B_vv"], t["dip"], order=2, device_ptrs=True,
                  store_amplitudes=0) as h:
        torch.cuda.synchronize()
        print(f"[fullsize] setup {time.time() - t0:.1f} s, device bytes {h.device_bytes() / 2**30:.1f} GiB, "
              f"E_MP2 {h.mp2_energy():.6f}", flush=True)
        t0 = time.time()
        h.products(U, out["A1"], out["B1"], out["S1"], order=1)
        h.products(U, out["A2"], out["B2"], out["S2"], order=2)
        torch.cuda.synchronize()
        print(f"[fullsize] products {time.time() - t0:.1f} s", flush=True)
        e2 = h.mp2_energy()
    assert e2 < 0.0
    Uh = U.cpu().numpy()
    r = {key: val.cpu().numpy() for key, val in out.items()}
    # first order: sampled rows (first and last row among them) against the row oracle
    rows = sorted({0, N - 1} | {int(x) for x in rng.choice(N, 6, replace=False)})
    t0 = time.time()
    eps = t["eps"].cpu().numpy()
    B_ov = t["B_ov"].cpu().numpy()
    Boo_i = [t["B_oo"][:, ia // v, :].cpu().numpy() for ia in rows]
    Bvv_a = [t["B_vv"][:, ia % v, :].cpu().numpy() for ia in rows]
    AV, BV = columns.first_order_rows(eps, o, v, B_ov, rows, Boo_i, Bvv_a, Uh)
    np.testing.assert_allclose(r["A1"][:, rows], AV, rtol=0, atol=1e-12 * np.abs(AV).max())
    np.testing.assert_allclose(r["B1"][:, rows], BV, rtol=0, atol=1e-12 * np.abs(BV).max())
    print(f"[fullsize] first-order rows {rows} ok ({time.time() - t0:.1f} s)", flush=True)
    if b2_rows:
        # complete second-order B rows from the element form
        t0 = time.time()
        B_oo = t["B_oo"].cpu().numpy()
        B_vv = t["B_vv"].cpu().numpy()
        sel = (rows[:1] + rows[3:5])[:b2_rows]
        _, BV2, _ = columns.second_order_rows(eps, o, v, B_oo, B_ov, B_vv, sel, Uh)
        del B_vv
        got = r["B2"][:, sel]
        np.testing.assert_allclose(got, BV2, rtol=0, atol=1e-12 * np.abs(BV2).max())
        part, part_ref = got - r["B1"][:, sel], BV2 - BV[:, [rows.index(x) for x in sel]]
        assert np.abs(part_ref).max() > 1e-7 * np.abs(BV2).max()
        np.testing.assert_allclose(part, part_ref, rtol=0, atol=1e-9 * np.abs(part_ref).max())
        print(f"[fullsize] second-order B rows {sel} ok ({time.time() - t0:.1f} s)", flush=True)
    np.testing.assert_allclose(r["S1"], Uh, rtol=0, atol=0)
    # second order: symmetric projections, a present and small correction
    for key in ("A2", "B2", "S2"):
        G = Uh @ r[key].T
        asym = np.abs(G - G.T).max()
        assert asym <= 1e-12 * np.abs(G).max(), (key, asym, np.abs(G).max())
    dA = np.linalg.norm(r["A2"] - r["A1"]) / np.linalg.norm(r["A1"])
    dB = np.linalg.norm(r["B2"] - r["B1"]) / np.linalg.norm(r["B1"])
    assert 1e-7 < dA < 0.1 and 1e-7 < dB < 0.5, (dA, dB)
    # S = 1 - (occupied and virtual MP2 densities): u^T S u < u^T u for every u
    q = np.einsum("kn,kn->k", Uh, r["S2"]) / np.einsum("kn,kn->k", Uh, Uh)
    assert np.all(q < 1.0) and np.all(q > 0.8), q


_ROW_ORACLE = {}


@pytest.mark.parametrize("store", [0, 1])
def test_mid_size_second_order_rows(P, store):
    """96/384/1152 (particle-hole dimension 36,864: many amplitude strips of 7 occupied
    rows with a ragged last one, interior 128 x 128 tiles, long C-index strides):
    sampled rows of the complete second-order A V, B V, S V against the row oracle with
    the MP2 densities, amplitudes rebuilt in strips or stored."""
    from synth import gen
    from oracle import columns
    t0 = time.time()
    sys_ = gen(9, 96, 384, 1152)
    o, v, N = sys_.o, sys_.v, sys_.N
    eps = np.concatenate([sys_.eps_o, sys_.eps_v])
    rng = np.random.default_rng(4)
    U = torch.tensor(rng.standard_normal((2, N)), device="cuda")
    out = {key: torch.empty_like(U) for key in ("A1", "B1", "S1", "A2", "B2", "S2")}
    print(f"[mid rows] store={store}: inputs {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    with P.Handle.from_system(sys_, order=2, store_amplitudes=store, strip_rows=7) as h:
        h.products(U, out["A1"], out["B1"], out["S1"], order=1)
        h.products(U, out["A2"], out["B2"], out["S2"], order=2)
        torch.cuda.synchronize()
    print(f"[mid rows] setup and products {time.time() - t0:.1f} s", flush=True)
    Uh = U.cpu().numpy()
    r = {key: val.cpu().numpy() for key, val in out.items()}
    t0 = time.time()
    rows = sorted({0, N - 1, 7 * v + 3} | {int(x) for x in rng.choice(N, 3, replace=False)})
    if "mid" not in _ROW_ORACLE:  # the same system and block in both modes: evaluate once
        dens = columns.mp2_densities(eps, o, v, sys_.B_ov)
        AV, BV, SV = columns.second_order_rows(eps, o, v, sys_.B_oo, sys_.B_ov, sys_.B_vv, rows, Uh, dens)
        AV1, BV1 = columns.first_order_rows(eps, o, v, sys_.B_ov, rows, [sys_.B_oo[:, ia // v, :] for ia in rows],
                                            [sys_.B_vv[:, ia % v, :] for ia in rows], Uh)
        _ROW_ORACLE["mid"] = (AV, BV, SV, AV1, BV1)
    AV, BV, SV, AV1, BV1 = _ROW_ORACLE["mid"]
    print(f"[mid rows] row oracle {time.time() - t0:.1f} s", flush=True)
    for key, ref, ref1 in (("A2", AV, AV1), ("B2", BV, BV1), ("S2", SV, Uh[:, rows])):
        got = r[key][:, rows]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max(), err_msg=key)
        np.testing.assert_allclose(r[key.replace("2", "1")][:, rows], ref1, rtol=0, atol=1e-12 * np.abs(ref1).max())
        part, part_ref = got - r[key.replace("2", "1")][:, rows], ref - ref1
        assert np.abs(part_ref).max() > 1e-7 * np.abs(ref).max(), key
        np.testing.assert_allclose(part, part_ref, rtol=0, atol=1e-9 * np.abs(part_ref).max(), err_msg=key)


def test_fullsize_fp32_products(P):
    """FP32 contractions (FP64 diagonal and assembly) against the FP64 path, amplitudes
    rebuilt in strips, at a size with several strips and GEMM tiles."""
    from synth.device_gen import gen_device
    o, v, X = 64, 256, 768
    t = gen_device(17, o, v, X)
    N = o * v
    rng = np.random.default_rng(3)
    U = torch.tensor(rng.standard_normal((4, N)), device="cuda")
    o64 = [torch.empty_like(U) for _ in range(3)]
    o32 = [torch.empty_like(U) for _ in range(3)]
    with P.Handle(t["eps"], t["B_oo"], t["B_ov"], t["B_vv"], t["dip"], order=2, device_ptrs=True,
                  store_amplitudes=0, strip_rows=5, precision=P.PP_FP32) as h:
        h.products(U, *o64, order=2, fp32=False)
        h.products(U, *o32, order=2, fp32=True)
    for j in range(3):
        a, b = o64[j].cpu().numpy(), o32[j].cpu().numpy()
        err = np.abs(a - b).max()
        assert err <= 2e-6 * np.abs(a).max(), (j, err, np.abs(a).max())
