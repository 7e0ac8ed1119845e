"""The serving loop (pp_server_*) through the C ABI.

Requests of differing systems, windows and root counts are solved together with
merged product passes; each result is checked against the oracle's exact pencil
solution, and against the same request solved alone on its own handle (the
result may not depend on what else was in the mix beyond the solver tolerance).
Admission by footprint, queueing, over-budget rejection and result delivery are
checked through the server's counters.
"""
import numpy as np
import pytest

from synth.gen import gen, gen_request
from oracle import dense, pencil

pytestmark = pytest.mark.gpu

# (seed, o, v, naux, omega0, n_roots): v = 4 o, naux = 12 o as in the serving stream
REQS = [(101, 6, 24, 72, 0.6, 5), (102, 8, 32, 96, 0.9, 6), (103, 5, 20, 60, 1.2, 4), (104, 7, 28, 84, 0.45, 6),
        (105, 9, 36, 108, 1.0, 8), (106, 6, 24, 72, 1.4, 4)]


@pytest.fixture(scope="module")
def P():
    import paper_2512_09811_amd as P
    P.lib()
    return P


def _systems():
    return [(gen(sd, o, v, x), w, nr) for sd, o, v, x, w, nr in REQS]


def _oracle(sys, w, nr):
    A, B, S = dense.assemble(sys, 2)
    e, X, Y, f = pencil.window_solve(A, B, S, sys.dip, w, nr)
    return e, f


def _check_vs(e, f, e_ref, f_ref, tol_e=1e-8):
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=tol_e)
    big = f_ref >= 1e-4 * f_ref.max()
    np.testing.assert_allclose(f[big], f_ref[big], rtol=1e-5)
    np.testing.assert_allclose(f[~big], f_ref[~big], rtol=0, atol=1e-9)


def test_server_mix_matches_oracle_and_solo(P):
    systems = _systems()
    print(f"[server] {len(systems)} requests, mixed sizes", flush=True)
    with P.Server(max_active=8) as srv:
        ids = [srv.submit_system(s, w, nr) for s, w, nr in systems]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == len(systems) and st["failed"] == 0
    # products of requests solving together were merged into shared passes
    assert st["passes"] > 0 and st["mean_requests_per_pass"] > 1.2, st
    assert st["peak_running"] >= 2
    print(f"[server] passes {st['passes']} grouped launches {st['grouped_launches']}", flush=True)
    assert st["peak_reserved_bytes"] <= st["budget_bytes"]
    assert 0 < st["latency_p50"] <= st["latency_p99"]
    for (s, w, nr), r in zip(systems, res):
        e_ref, f_ref = _oracle(s, w, nr)
        _check_vs(r["energies"], r["osc"], e_ref, f_ref)
        assert np.all(r["converged"] == 1) and r["status"] == P.PP_OK
        with P.Handle.from_system(s, order=2) as h:
            e1, v1, f1, _ = h.window_solve(w, nr)
        np.testing.assert_allclose(r["energies"], e1, rtol=0, atol=1e-9)
        np.testing.assert_allclose(r["osc"], f1, rtol=1e-6, atol=1e-12)
        # eigenvectors: same up to sign (non-degenerate roots)
        for q in range(nr):
            ov = abs(float(np.dot(r["vectors"][q].ravel(), v1[q].ravel())))
            nn = np.linalg.norm(r["vectors"][q]) * np.linalg.norm(v1[q])
            assert abs(ov / nn - 1.0) < 1e-6


def test_server_admission_by_footprint(P):
    """A budget that holds one request at a time: requests queue and run one by one."""
    systems = _systems()[:3]
    with P.Server(max_active=8) as probe:
        need = [probe.request_bytes(s.o, s.v, s.naux, nr) for s, w, nr in systems]
    budget = max(need) + min(need) // 2
    print(f"[server] admission budget {budget} B, footprints {need}", flush=True)
    with P.Server(hbm_budget=budget, max_active=8) as srv:
        ids = [srv.submit_system(s, w, nr) for s, w, nr in systems]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == 3 and st["peak_running"] == 1
    assert st["peak_reserved_bytes"] <= budget
    assert res[2]["queued_seconds"] > 0.0
    for (s, w, nr), r in zip(systems, res):
        e_ref, f_ref = _oracle(s, w, nr)
        _check_vs(r["energies"], r["osc"], e_ref, f_ref)


def test_server_rejects_and_delivers_once(P):
    s, w, nr = _systems()[0]
    with P.Server(max_active=2) as probe:
        need = probe.request_bytes(s.o, s.v, s.naux, nr)
    with P.Server(hbm_budget=need // 2) as srv:
        with pytest.raises(P.PPError) as ei:
            srv.submit_system(s, w, nr)
        assert ei.value.status == P.PP_ENOMEM
    with P.Server() as srv:
        bad = gen(1, 4, 16, 48)
        bad.B_ov[0, 0, 0] = np.inf
        with pytest.raises(P.PPError) as ei:
            srv.submit_system(bad, 0.5, 3)
        assert ei.value.status == P.PP_EINVAL
        rid = srv.submit_system(s, w, nr)
        r = None
        import time
        t0 = time.time()
        while r is None and time.time() - t0 < 60:
            r = srv.poll(rid)
            time.sleep(0.01)
        assert r is not None and r["status"] == P.PP_OK
        with pytest.raises(KeyError):
            srv.poll(rid)


@pytest.mark.parametrize("prec", ["fp32", "sbf16"])
def test_server_mixed_precision(P, prec):
    """FP32 contractions (the amplitude one as split-BF16 products in sbf16 mode) with FP64
    refinement inside the server meet the FP64 bar."""
    systems = _systems()[:4]
    with P.Server(precision=P.PP_FP32 if prec == "fp32" else P.PP_SPLIT_BF16) as srv:
        ids = [srv.submit_system(s, w, nr) for s, w, nr in systems]
        res = [srv.wait(i) for i in ids]
    for (s, w, nr), r in zip(systems, res):
        e_ref, f_ref = _oracle(s, w, nr)
        _check_vs(r["energies"], r["osc"], e_ref, f_ref)
        assert np.all(r["residual"] <= 1e-9)


def test_server_stream_shape(P):
    """Requests drawn like the serving stream (smaller occupied range): all converge."""
    reqs = [gen_request(r, 8, 16) for r in range(6)]
    with P.Server() as srv:
        ids = [srv.submit_system(s, w, nr) for s, w, nr in reqs]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == 6
    for (s, w, nr), r in zip(reqs, res):
        assert r["n_roots"] == nr and np.all(r["converged"] == 1)
        assert np.all(np.diff(r["energies"]) >= 0)


def test_server_riesz_requests(P):
    """A server whose requests use the Riesz-projector window solve: results match the
    oracle, and the requests' contour solves share product passes."""
    systems = _systems()[:3]
    print(f"[server riesz] {len(systems)} requests", flush=True)
    with P.Server(max_active=4, method=P.PP_RIESZ) as srv:
        ids = [srv.submit_system(s, w, nr) for s, w, nr in systems]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == len(systems) and st["failed"] == 0
    for (s, w, nr), r in zip(systems, res):
        e_ref, f_ref = _oracle(s, w, nr)
        _check_vs(r["energies"], r["osc"], e_ref, f_ref)
        assert np.all(r["converged"] == 1) and r["status"] == P.PP_OK


def _request_golden():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "serve_o40_v160_x480.json")))


@pytest.mark.parametrize("prec", ["fp64", "sbf16"])
def test_server_o40_request_alone_and_in_mix(P, prec):
    """A request of the serving stream's shape at n_occ = 40 (n_vir 160, n_aux 480; its
    roots stored from the oracle's exact pencil solution) served alone, then in a mix with
    smaller requests whose products share its passes: the same roots and strengths both
    times, to the FP64 bar also when the subspace is built from split-BF16 products."""
    g = _request_golden()
    big = gen(g["seed"], g["o"], g["v"], g["naux"])
    e_ref, f_ref = np.array(g["energies"]), np.array(g["osc"])
    pp = {"fp64": P.PP_FP64, "sbf16": P.PP_SPLIT_BF16}[prec]
    print(f"[server o40] {prec}: alone", flush=True)
    with P.Server(precision=pp) as srv:
        r = srv.wait(srv.submit_system(big, g["omega0"], g["n_roots"]))
    _check_vs(r["energies"], r["osc"], e_ref, f_ref)
    assert np.all(r["converged"] == 1) and np.all(r["residual"] <= 1e-8)
    print(f"[server o40] {prec}: in a mix", flush=True)
    mix = _systems()[:3]
    with P.Server(precision=pp, max_active=8) as srv:
        ids = [srv.submit_system(s, w, nr) for s, w, nr in mix[:2]]
        ib = srv.submit_system(big, g["omega0"], g["n_roots"])
        ids.append(srv.submit_system(*mix[2]))
        rb = srv.wait(ib)
        rs = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == 4 and st["failed"] == 0 and st["peak_running"] >= 2
    _check_vs(rb["energies"], rb["osc"], e_ref, f_ref)
    np.testing.assert_allclose(rb["energies"], r["energies"], rtol=0, atol=1e-9)
    for (s, w, nr), q in zip(mix[:2] + mix[2:], rs):
        e1, f1 = _oracle(s, w, nr)
        _check_vs(q["energies"], q["osc"], e1, f1)


def test_server_results_do_not_depend_on_the_mix(P):
    """A request's products do not depend on which requests share its passes: the o = 40
    request served alone and then beside an o = 24 request (large enough that their GEMMs
    go out as grouped launches) and a small one gives bitwise equal roots, strengths and
    vectors (no GEMM of a merged pass takes split-K, grouped or launched alone)."""
    g = _request_golden()
    big = gen(g["seed"], g["o"], g["v"], g["naux"])
    mid = gen(4041, 24, 96, 288)
    print("[server mix] alone", flush=True)
    with P.Server(max_active=8) as srv:
        alone = srv.wait(srv.submit_system(big, g["omega0"], g["n_roots"]))
    print("[server mix] in a mix", flush=True)
    with P.Server(max_active=8) as srv:
        ids = [srv.submit_system(mid, 0.7, 6), srv.submit_system(big, g["omega0"], g["n_roots"]),
               srv.submit_system(*_systems()[0])]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["peak_running"] >= 2 and st["grouped_launches"] > 0, st
    mixed = res[1]
    assert np.array_equal(alone["energies"], mixed["energies"])
    assert np.array_equal(alone["osc"], mixed["osc"])
    assert np.array_equal(alone["vectors"], mixed["vectors"])
    _check_vs(mixed["energies"], mixed["osc"], np.array(g["energies"]), np.array(g["osc"]))
