"""Benchmark: the second-order product on one MI355X.

Default workload (one "step"): the largest matrix-free second-order system, n_occ =
256, n_vir = 1024, n_aux = 4096 (particle-hole dimension 262,144, amplitudes never
stored), inputs resident in HBM.  A product pass M X over m = 8 trial 2N-vectors (16
particle-hole vectors: the largest batch whose FP32 intermediates fit beside the
operands) is issued as 16 parts of 16 occupied rows (pp_sigma_part); one step is one
part: the amplitude strips of its rows are rebuilt from B^ov and the orbital-energy
denominators (split-BF16 integrals, FP32 strip, in-place split), multiplied into H = tau G
(split-BF16 products) and contracted into the output, nothing hoisted.  Part 0 of every
pass also runs the pass prologue (first-order terms, G = V B^vv - B^oo V and its split,
delta-type terms) and the last part the FP64 assembly, so 16 steps are one whole pass.
Precision: contractions in FP32 with the amplitude ones as split-BF16 products (the
mixed-precision form); the FP64 path is timed beside it on the same step (8 trial
vectors' worth of memory only allows 4 2N-vectors there), and one complete reduced pass
is compared with the FP64 pass on the same vectors.

value = sigma-build TFLOP/s (algorithmic flops of the parts timed / wall time).  The
40/160/600 window solves (solves/s at 1e-6 Ha against the oracle, FP64 and split-BF16,
p50/p99 latency) are reported as extra fields.  ``--workload mp2_o40_v160_x600`` gives
that window benchmark as its own line; ``--large mp2_o200_v800_x3000`` a window of a
device-drawn large system in split BF16 and FP64 with the roots cross-checked; ``--serve``
the serving stream; ``--riesz`` the Riesz-projector comparison.

Prints ONE JSON line (rank 0): roofline of the dominant kernel (the amplitude
contraction, split-BF16, priced against the BF16 peak / 3) and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
# split BF16: three BF16 MFMA products (dense 2.5 PFLOP/s) per FP32-equivalent product
PEAK_SPLIT_BF16_TFLOPS = 2500.0 / 3.0
PRECISIONS = {"fp64": 0, "fp32": 1, "sbf16": 2}
DTYPES = {"fp64": "f64", "fp32": "f32", "sbf16": "bf16x3"}
HBM_TBPS = 8.0

# HBM traffic of the amplitude contraction H = tau G at this workload (FP64, 4
# windows), per launch, from two rocprofv3 --pmc runs of this script (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch) scaled by what the same counters read for a
# plain 1 GiB device copy in the same runs (--copy-calibration).  The figures hold
# for the GEMM source with this digest and for launches of this size only;
# otherwise the roofline reports traffic as null.
HHAT_TRAFFIC = {"gemm_sha256_16": "b19e12b0544abbee", "flops_per_launch": 1629577846153.8462,
                "fetch_kib": 11596260.0, "write_kib": 1004216.1,
                "copy_fetch_kib": 524310.0, "copy_write_kib": 1048576.0}


def hhat_traffic(flops_per_launch, precision):
    """Calibrated HBM bytes per launch of the amplitude contraction, or None."""
    import hashlib
    src = os.path.join(ROOT, "paper_2512_09811_amd", "csrc", "gemm.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    t = HHAT_TRAFFIC
    if precision != "fp64" or digest != t["gemm_sha256_16"] or abs(flops_per_launch / t["flops_per_launch"] - 1) > 1e-9:
        return None
    kib = 1 << 20  # KiB in a GiB
    fetch = t["fetch_kib"] * (kib / t["copy_fetch_kib"])
    write = t["write_kib"] * (kib / t["copy_write_kib"])
    return 1024.0 * (fetch + write)


# HBM traffic of the split-BF16 amplitude contraction of the product benchmark, per
# launch, from two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch) scaled by what the same counters read for a plain 1 GiB device copy
# in the same runs (--copy-calibration); valid for the GEMM source with this digest and
# launches of this size only (else null).
PRODUCT_TRAFFIC = {"gemm_sha256_16": "10c6f2ce9ca92a7d", "flops_per_launch": 281474976710656.0,
                   "fetch_kib": 402842875.0, "write_kib": 2392064.0,
                   "copy_fetch_kib": 524303.6, "copy_write_kib": 1048576.0}


def product_traffic(flops_per_launch):
    """Calibrated HBM bytes per launch of the product benchmark's amplitude GEMM, or None."""
    import hashlib
    t = PRODUCT_TRAFFIC
    if t is None:
        return None
    src = os.path.join(ROOT, "paper_2512_09811_amd", "csrc", "gemm.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    if digest != t["gemm_sha256_16"] or abs(flops_per_launch / t["flops_per_launch"] - 1) > 1e-9:
        return None
    kib = 1 << 20
    return 1024.0 * (t["fetch_kib"] * (kib / t["copy_fetch_kib"]) + t["write_kib"] * (kib / t["copy_write_kib"]))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mp2_o256_v1024_x4096",
                    help="mp2_o256_v1024_x4096: the product benchmark (default); mp2_o40_v160_x600 (or another "
                         "workload with stored oracle values): window solves")
    ap.add_argument("--precision", choices=list(PRECISIONS), default=None,
                    help="product benchmark: sbf16 (default) or fp32; window solves: fp64 (default), fp32, sbf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-windows", action="store_true",
                    help="product benchmark: skip the 40/160/600 window solves reported beside it")
    ap.add_argument("--no-fp64", action="store_true",
                    help="product benchmark: skip the FP64 figure and the reduced-vs-FP64 check (profiling runs)")
    ap.add_argument("--tol", type=float, default=1e-8,
                    help="solver residual tolerance; every timed window is still checked against the oracle "
                         "(1e-6 Ha, 1e-5 relative f) and only windows that pass count")
    ap.add_argument("--windows", type=int, default=0, help="use only the first N windows (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three plain 1 GiB device copies (reference dispatches for HBM traffic counters)")
    ap.add_argument("--serve", action="store_true",
                    help="serving stream instead of the batched-window workload (its own JSON line)")
    ap.add_argument("--requests", type=int, default=24, help="serving: timed requests")
    ap.add_argument("--occ", default="16,64", help="serving: n_occ range lo,hi (the full stream is 16,128)")
    ap.add_argument("--no-plain-compare", action="store_true",
                    help="serving: skip solving the timed requests one by one on plain FP64 handles")
    ap.add_argument("--riesz", action="store_true",
                    help="Riesz-projector windows against folded inverse-Krylov windows on the same small and "
                         "mid-size systems (its own JSON line)")
    ap.add_argument("--large", default=None, metavar="WORKLOAD",
                    help="window solves of a system drawn on the device (mp2_o200_v800_x3000 or "
                         "mp2_o256_v1024_x4096, amplitudes rebuilt in strips) in each precision of "
                         "--large-precisions, roots cross-checked between them (its own JSON line)")
    ap.add_argument("--large-precisions", default="sbf16,fp64")
    ap.add_argument("--large-roots", type=int, default=4)
    ap.add_argument("--large-omega", type=float, default=0.3)
    return ap.parse_args()


def cpu_baseline(name):
    """The FP64 oracle on the host cores: dense assembly + exact diagonalisation of the
    same system, one diagonalisation serving every window of the workload."""
    from synth.gen import CONFIGS, WINDOWS, gen_config
    from oracle import dense, pencil
    cfg = CONFIGS[name]
    omegas, nr = WINDOWS[name]
    sys_ = gen_config(name)
    t0 = time.perf_counter()
    A, B, S = dense.assemble(sys_, cfg["order"])
    om, X, Y = pencil.solve_all(A, B, S)
    for w0 in omegas:
        idx = pencil.select_window(om, float(w0), nr)
        pencil.oscillator_strengths(om[idx], X[:, idx], Y[:, idx], sys_.dip)
    dt = time.perf_counter() - t0
    try:
        import threadpoolctl
        threads = max((p.get("num_threads", 0) for p in threadpoolctl.threadpool_info()), default=0)
    except Exception:
        threads = 0
    cores = threads or os.cpu_count()
    return dict(value=len(omegas) / dt, unit="solves/s", cores=int(cores), kind="oracle",
                sample=f"dense oracle on the full workload: assembly of A, B, S (N = {sys_.N}) and exact pencil "
                       f"diagonalisation, one diagonalisation serving all {len(omegas)} windows; {dt:.1f} s")


# Riesz-projector comparison: (name, n_occ, n_vir, n_aux, order, seed, windows, roots)
RIESZ_WORKLOADS = [("rpa1_o8_v24_x64", 8, 24, 64, 1, 1, [0.5], 6),
                   ("mp2_o16_v64_x192", 16, 64, 192, 2, 6, [0.4, 0.8], 8)]


def riesz_main(args):
    """Window solves by the Riesz projector (contour-filtered subspace iteration) and by
    the folded inverse-Krylov method on the same systems, each window checked against
    the oracle; solves/s over the timed repetitions of each batch of windows."""
    import torch  # noqa: F401  (initializes the device runtime first)
    import paper_2512_09811_amd as P
    from synth.gen import gen
    from oracle import dense, pencil
    results = []
    for name, o, v, naux, order, seed, oms, nr in RIESZ_WORKLOADS:
        sys_ = gen(seed, o, v, naux)
        A, B, S = dense.assemble(sys_, order)
        ref = [pencil.window_solve(A, B, S, sys_.dip, w, nr) for w in oms]
        for method in ("folded", "riesz"):
            m = P.PP_RIESZ if method == "riesz" else P.PP_FOLDED
            with P.Handle.from_system(sys_, order=order, method=m, tol=args.tol) as h:
                h.window_solve_batch(oms, nr)                       # warm-up
                t0 = time.perf_counter()
                for _ in range(max(1, args.steps)):
                    E, V, F, infos = h.window_solve_batch(oms, nr)
                dt = (time.perf_counter() - t0) / max(1, args.steps)
            de = max(float(np.abs(E[w] - ref[w][0]).max()) for w in range(len(oms)))
            df = 0.0
            ok = 0
            for w in range(len(oms)):
                fr = ref[w][3]
                big = fr >= 1e-4 * fr.max()
                rel = float(np.max(np.abs(F[w][big] - fr[big]) / fr[big])) if big.any() else 0.0
                df = max(df, rel)
                ok += int(np.abs(E[w] - ref[w][0]).max() <= 1e-6 and rel <= 1e-5)
            results.append(dict(workload=name, method=method, value=ok / dt, unit="solves/s",
                                seconds_per_batch=dt, windows=len(oms), n_roots=nr,
                                windows_meeting_tolerance=f"{ok}/{len(oms)}",
                                products_per_window=float(np.mean([i["products"] for i in infos])),
                                cycles_per_window=float(np.mean([i["cycles"] for i in infos])),
                                max_abs_dE_ha=de, max_rel_df=df))
            print(f"[riesz] {name} {method}: {ok / dt:.2f} solves/s, "
                  f"{results[-1]['products_per_window']:.0f} products/window", file=sys.stderr, flush=True)
    print(json.dumps(dict(metric="window solves/s, Riesz projector vs folded inverse Krylov", unit="solves/s",
                          dtype="f64", data="synthetic (seeded generator)", solver_tol=args.tol,
                          results=results)), flush=True)


def large_main(args):
    """Window solves at the sizes where no dense oracle fits (amplitudes rebuilt in strips
    every pass): one window per precision on a system drawn on the device, each on its own
    handle (setup untimed), the roots of the reduced-precision solve checked against the
    FP64 solve's at 1e-6 Ha and 1e-5 relative f; solves/s, products and sigma-build
    TFLOP/s per precision."""
    import torch
    import paper_2512_09811_amd as P
    from synth.device_gen import gen_device
    from synth.gen import CONFIGS

    name = args.large
    cfg = CONFIGS[name]
    P.lib()
    t = gen_device(cfg["seed"], cfg["o"], cfg["v"], cfg["naux"])
    torch.cuda.synchronize()
    w0, nr = args.large_omega, args.large_roots
    runs = {}
    for pn in args.large_precisions.split(","):
        t0 = time.perf_counter()
        with P.Handle(t["eps"], t["B_oo"], t["B_ov"], t["B_vv"], t["dip"], order=2, device_ptrs=True,
                      precision=PRECISIONS[pn], store_amplitudes=0, tol=args.tol) as h:
            setup = time.perf_counter() - t0
            print(f"[large] {name} {pn}: setup {setup:.1f} s", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, _, f, info = h.window_solve(w0, nr, vectors=False, allow_unconverged=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = h.stats()
        runs[pn] = dict(seconds=dt, solves_per_s=1.0 / dt, setup_seconds=setup, products=int(info["products"]),
                        cycles=int(info["cycles"]), converged=int(np.sum(info["converged"])),
                        max_residual=float(np.max(info["residual"])),
                        sigma_tflops=st["product_flops"] / st["product_seconds"] / 1e12 if st["product_seconds"] else 0.0,
                        amplitude_gemm_tflops=st["hhat_flops"] / st["hhat_seconds"] / 1e12 if st["hhat_seconds"] else 0.0,
                        sigma_fraction_of_time=st["product_seconds"] / dt,
                        energies=[float(x) for x in e], osc=[float(x) for x in f])
        if pn == "fp64":
            runs[pn]["amplitude_gemm_frac_of_fp64_peak"] = runs[pn]["amplitude_gemm_tflops"] / PEAK_FP64_MFMA_TFLOPS
        else:
            # the amplitude-GEMM figures of a mixed solve cover its reduced-precision launches
            # and the FP64 launches of its refinement together
            runs[pn]["amplitude_gemm_note"] = ("reduced-precision and FP64 refinement launches together; the "
                                               "split-BF16 kernel alone is measured by the default product line")
        print(f"[large] {name} {pn}: {dt:.1f} s, {info['products']} products, residual {np.max(info['residual']):.1e}",
              file=sys.stderr, flush=True)
    names = list(runs)
    check = {}
    if "fp64" in runs:
        ref = runs["fp64"]
        ge, gf = np.array(ref["energies"]), np.array(ref["osc"])
        for pn in names:
            if pn == "fp64":
                continue
            e, f = np.array(runs[pn]["energies"]), np.array(runs[pn]["osc"])
            big = gf >= 1e-4 * gf.max()
            de = float(np.abs(e - ge).max())
            df = float(np.max(np.abs(f[big] - gf[big]) / gf[big]))
            check[pn] = dict(max_abs_dE_ha=de, max_rel_df=df, within_1e6_ha_1e5_f=bool(de <= 1e-6 and df <= 1e-5))
    first = runs[names[0]]
    line = {
        "metric": "window solves/sec + sigma-build TFLOP/s at 1e-6 Ha; p50/p99 solve latency",
        "value": first["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": 1e3 * first["seconds"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[names[0]],
        "data": "synthetic (seeded device generator; PbS/CdS orbitals and integrals are not available)",
        "config": {"workload": f"{name}: second-order window solve, n_occ={cfg['o']}, n_vir={cfg['v']}, "
                               f"n_aux={cfg['naux']}, 1 window at {w0} Ha x {nr} roots, amplitudes rebuilt in strips",
                   "solver_tol": args.tol, "precisions": names, "parallelism": "single GPU"},
        "runs": runs,
        "reduced_vs_fp64": check,
    }
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    print(json.dumps(line), flush=True)


def serve_main(args):
    """Serving stream: requests drawn like the serving workload (n_vir = 4 n_occ,
    n_aux = 12 n_occ, omega0 ~ U[0.3, 1.5], 4-12 roots), submitted to one pp_server.
    Every request is solved to the window benchmark's tolerance (--tol).  After a short
    warm-up (runtime start), the timed requests are first submitted all at once to a fresh
    server: their completion rate is the saturated throughput X.  The same
    requests then arrive as a Poisson process at 0.8 X (the timed stream: value, latency
    from submission to result).  Last, the plain path: one FP64 handle per request, one
    request at a time."""
    import threading
    import torch  # noqa: F401  (initializes the device runtime first)
    import paper_2512_09811_amd as P
    from synth.gen import gen_request
    lo, hi = (int(x) for x in args.occ.split(","))
    prec = PRECISIONS[args.precision or "fp64"]
    nwarm = 4
    t0 = time.perf_counter()
    reqs = [gen_request(r, lo, hi) for r in range(nwarm + args.requests)]
    print(f"[serve] generated {len(reqs)} requests in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    timed = reqs[nwarm:]
    with P.Server(precision=prec, tol=args.tol) as srv:
        ids = [srv.submit_system(s_, w, nr) for s_, w, nr in reqs[:nwarm]]
        for i in ids:
            srv.wait(i, allow_unconverged=True)
    print("[serve] warm-up done", file=sys.stderr, flush=True)
    # saturated: every timed request at once
    t1 = time.perf_counter()
    with P.Server(precision=prec, tol=args.tol) as srv2:
        ids2 = [srv2.submit_system(s_, w, nr) for s_, w, nr in timed]
        for j, i in enumerate(ids2):
            srv2.wait(i, allow_unconverged=True)
            if (j + 1) % 8 == 0:
                print(f"[serve] saturated {j + 1}/{len(ids2)}", file=sys.stderr, flush=True)
        st2 = srv2.stats()
    x_sat = len(timed) / (time.perf_counter() - t1)
    lam = 0.8 * x_sat
    print(f"[serve] saturated {x_sat:.2f} solves/s ({st2['mean_requests_per_pass']:.2f} requests per pass); "
          f"arrivals at {lam:.2f}/s", file=sys.stderr, flush=True)
    srv = P.Server(precision=prec, tol=args.tol)
    rng = np.random.default_rng(12345)
    gaps = rng.exponential(1.0 / lam, args.requests)
    ids = [None] * len(timed)

    def client():
        t_next = time.perf_counter()
        for j, (s_, w, nr) in enumerate(timed):
            t_next += gaps[j]
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            ids[j] = srv.submit_system(s_, w, nr)

    t0 = time.perf_counter()
    th = threading.Thread(target=client)
    th.start()
    th.join()
    res = []
    for j, i in enumerate(ids):
        res.append(srv.wait(i, allow_unconverged=True))
        if (j + 1) % 8 == 0:
            print(f"[serve] {j + 1}/{len(ids)} results", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    conv = sum(1 for r in res if r["status"] == P.PP_OK and np.all(r["converged"] == 1))
    seq = None
    if not args.no_plain_compare:
        t1 = time.perf_counter()
        for j, (s_, w, nr) in enumerate(timed):
            with P.Handle.from_system(s_, order=2, tol=args.tol) as h:
                h.window_solve(w, nr, allow_unconverged=True)
            if (j + 1) % 8 == 0:
                print(f"[serve] plain path {j + 1}/{len(timed)}", file=sys.stderr, flush=True)
        seq = len(timed) / (time.perf_counter() - t1)
    lat = np.array([r["latency_seconds"] for r in res])
    occ = [s_.o for s_, _, _ in timed]
    line = {
        "metric": "serving: window solves/sec with p50/p99 latency (Poisson arrivals at 0.8x saturated rate)",
        "value": conv / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": nwarm,
        "ms_per_step": 1e3 * elapsed / args.requests,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision or "fp64"],
        "data": "synthetic (seeded serving stream)",
        "config": {"workload": f"serving stream: {args.requests} requests, n_occ ~ U{{{lo}..{hi}}}, n_vir = 4 n_occ, "
                               f"n_aux = 12 n_occ, omega0 ~ U[0.3,1.5], 4-12 roots, second order",
                   "arrival_rate_per_s": lam, "mean_n_occ": float(np.mean(occ)), "solver_tol": args.tol},
        "windows_converged": f"{conv}/{len(res)}",
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "queued_p50_s": st["queued_p50"],
        "queued_p99_s": st["queued_p99"],
        "passes": st["passes"],
        "mean_requests_per_pass": st["mean_requests_per_pass"],
        "grouped_launches": st["grouped_launches"],
        "peak_running": st["peak_running"],
        "sigma_tflops": st["product_flops"] / st["product_seconds"] / 1e12 if st["product_seconds"] > 0 else 0.0,
        "sigma_fraction_of_time": st["product_seconds"] / elapsed,
        "saturated_solves_per_s": x_sat,
        "saturated_requests_per_pass": st2["mean_requests_per_pass"],
        "plain_fp64_one_at_a_time_solves_per_s": seq,
        "saturated_over_plain": (x_sat / seq) if seq else None,
    }
    print(json.dumps(line), flush=True)


def windows_run(args, name, precision_name, steps, warmup, cpu):
    """Window solves of one workload (all its windows in one batched call per step: setup,
    solves, teardown), checked against the stored oracle values; returns the JSON line."""
    import torch
    import paper_2512_09811_amd as P
    from synth.gen import CONFIGS, WINDOWS, gen_config

    P.lib()
    cfg = CONFIGS[name]
    omegas, nr = WINDOWS[name]
    if args.windows:
        omegas = omegas[: args.windows]
    sys_ = gen_config(name)
    dev = torch.device("cuda:0")
    t = {k: torch.tensor(getattr(sys_, k), dtype=torch.float64, device=dev).contiguous()
         for k in ("eps", "B_oo", "B_ov", "B_vv", "dip")}
    torch.cuda.synchronize()
    precision = PRECISIONS[precision_name]
    golden_path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    golden = json.load(open(golden_path)) if os.path.exists(golden_path) else None

    def step(record):
        h = P.Handle(t["eps"], t["B_oo"], t["B_ov"], t["B_vv"], t["dip"], order=cfg["order"], device_ptrs=True,
                     precision=precision, store_amplitudes=1, tol=args.tol)
        res = []
        t0 = time.perf_counter()
        E, VEC, F, INFOS = h.window_solve_batch([float(w) for w in omegas], nr, vectors=True, osc=True,
                                                allow_unconverged=True)
        for k, w0 in enumerate(omegas):
            # latency of a window = wall time of its own solver thread (arrival at the
            # batch call to its last output), reported by the library
            res.append((float(w0), E[k], F[k], INFOS[k], INFOS[k]["seconds"]))
        st = h.stats()
        h.close()
        if record is not None:
            record.append((res, st))
        return res

    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(recs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    lat = [r[4] for res, _ in recs for r in res]
    prod_flops = sum(st["product_flops"] for _, st in recs)
    prod_sec = sum(st["product_seconds"] for _, st in recs)
    h_flops = sum(st["hhat_flops"] for _, st in recs)
    h_sec = sum(st["hhat_seconds"] for _, st in recs)
    h_n = sum(st["hhat_launches"] for _, st in recs)
    # accuracy against the stored oracle values
    max_de, max_df, ok = 0.0, 0.0, 0
    total = 0
    for res, _ in recs:
        for k, (w0, e, f, info, _) in enumerate(res):
            total += 1
            if golden is None:
                continue
            g = golden["windows"][k]
            ge, gf = np.array(g["energies"]), np.array(g["osc"])
            de = float(np.abs(e - ge).max())
            big = gf >= 1e-4 * gf.max()
            df = float(np.max(np.abs(f[big] - gf[big]) / gf[big])) if big.any() else 0.0
            dfs = float(np.max(np.abs(f[~big] - gf[~big]))) if (~big).any() else 0.0
            max_de, max_df = max(max_de, de), max(max_df, df)
            if de <= 1e-6 and df <= 1e-5 and dfs <= 1e-9 and info["status"] == P.PP_OK:
                ok += 1
    n_windows = len(omegas) * steps
    value = ok / elapsed if golden is not None else n_windows / elapsed
    peak = {"fp64": PEAK_FP64_MFMA_TFLOPS, "fp32": PEAK_FP32_MFMA_TFLOPS, "sbf16": PEAK_SPLIT_BF16_TFLOPS}[precision_name]
    achieved = (h_flops / h_sec) / 1e12 if h_sec > 0 else 0.0
    # algorithmic bytes of one launch: tau (N x N) read once, G read and H written once
    kX = (h_flops / max(h_n, 1)) / (2.0 * cfg["o"] * cfg["v"] * cfg["o"] * cfg["v"])
    Nph = cfg["o"] * cfg["v"]
    hhat_bytes = 8.0 * Nph * Nph + 16.0 * Nph * kX
    line = {
        "metric": "window solves/sec + sigma-build TFLOP/s at 1e-6 Ha; p50/p99 solve latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[precision_name],
        "data": "synthetic (seeded generator; PbS/CdS orbitals and integrals are not available)",
        "config": {"workload": f"{name}: second-order, n_occ={cfg['o']}, n_vir={cfg['v']}, n_aux={cfg['naux']}, "
                               f"{len(omegas)} windows x {nr} roots, amplitudes stored",
                   "windows_ha": [float(x) for x in omegas], "n_roots": nr, "solver_tol": args.tol,
                   "parallelism": "single GPU"},
        "windows_meeting_tolerance": f"{ok}/{total}" if golden is not None else "unchecked",
        "max_abs_dE_ha": max_de,
        "max_rel_df": max_df,
        "sigma_tflops": (prod_flops / prod_sec) / 1e12 if prod_sec > 0 else 0.0,
        "sigma_fraction_of_time": prod_sec / elapsed,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "products_per_window": float(np.mean([r[3]["products"] for res, _ in recs for r in res])),
        "roofline": {"bound": "mfma",
                     "kernel": ("gemm_kernel<double,128,128,16,1> (H = tau G; a call is the main launch plus a "
                                "peeled 64x64 tail when its last wave would run at most half full)"
                                if precision_name == "fp64" else
                                "gemm_kernel<float,128,128,16,1> and its FP64 refinement passes (H = tau G), "
                                "priced against the FP32 peak"
                                if precision_name == "fp32" else
                                "gemm_sbf16_kernel (split BF16, three BF16 MFMAs per product) and its FP64 "
                                "refinement passes (H = tau G), priced against the BF16 peak / 3"),
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "launches": h_n, "avg_launch_ms": 1e3 * h_sec / max(h_n, 1),
                     "flops_per_launch": h_flops / max(h_n, 1),
                     "traffic": hhat_traffic(h_flops / max(h_n, 1), precision_name),
                     "algorithmic_bytes_per_launch": hhat_bytes},
    }
    if args.copy_calibration:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the
        # traffic counters of the kernels above (1 GiB = 1048576 KiB each way)
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if cpu:
        line["cpu_baseline"] = cpu_baseline(name)
    return line




# The default workload: the largest matrix-free second-order system, products in parts.
PRODUCT_WORKLOAD = "mp2_o256_v1024_x4096"
PRODUCT_M = 8           # trial 2N-vectors per reduced-precision pass (16 particle-hole vectors)
PRODUCT_M_FP64 = 4      # FP64 pass width (FP64 intermediates take twice the memory)
PRODUCT_PARTS = 16      # parts per pass: 16 occupied rows each (one step = one part)
PRODUCT_STRIP_ROWS = 8  # occupied rows per amplitude strip (two strips per part)


def product_cpu_baseline(o, v, X, seed, k, flops_per_row):
    """The oracle's rows of the same product on the host cores: one row of the complete
    second-order B V and of the first-order A V for k vectors (oracle.columns, the
    element form), from host copies of the same device-drawn inputs.  Reported in the
    metric's unit: the algorithmic flops of the rows computed (the pass's flops per
    particle-hole row) per second of oracle time."""
    import torch
    from synth.device_gen import gen_device
    from oracle import columns
    t = gen_device(seed, o, v, X)
    host = {key: val.cpu().numpy() for key, val in t.items()}
    del t
    torch.cuda.empty_cache()
    eps = host["eps"]
    rng = np.random.default_rng(7)
    V = rng.standard_normal((k, o * v))
    row = int(rng.integers(o * v))
    t0 = time.perf_counter()
    columns.second_order_rows(eps, o, v, host["B_oo"], host["B_ov"], host["B_vv"], [row], V)
    dt = time.perf_counter() - t0
    try:
        import threadpoolctl
        threads = max((p.get("num_threads", 0) for p in threadpoolctl.threadpool_info()), default=0)
    except Exception:
        threads = 0
    return dict(value=flops_per_row / dt / 1e12, unit="TFLOP/s", cores=int(threads or os.cpu_count()),
                kind="oracle",
                sample=f"one particle-hole row ({row}) of the complete second-order B V and first-order A V for "
                       f"{k} vectors by the row oracle (element form; the delta-type A and S rows, which need the "
                       f"MP2 densities, left out), {dt:.1f} s; scaled by the pass's algorithmic flops per row, "
                       f"{flops_per_row:.3e}")


def product_main(args):
    """The default benchmark line (see the module docstring)."""
    import torch
    import paper_2512_09811_amd as P
    from synth.gen import CONFIGS
    from synth.device_gen import gen_device
    P.lib()
    cfg = CONFIGS[PRODUCT_WORKLOAD]
    o, v, X, seed = cfg["o"], cfg["v"], cfg["naux"], cfg["seed"]
    N = o * v
    prec_name = args.precision or "sbf16"
    if prec_name == "fp64":
        raise SystemExit("the product benchmark's headline is the reduced-precision pass; FP64 is timed beside it")
    budget = int(torch.cuda.get_device_properties(0).total_memory - (6 << 30))

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def make_handle(precision):
        t = gen_device(seed, o, v, X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = P.Handle(t["eps"], t["B_oo"], t["B_ov"], t["B_vv"], t["dip"], order=2, device_ptrs=True,
                     precision=precision, store_amplitudes=0, strip_rows=PRODUCT_STRIP_ROWS, hbm_budget=budget)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del t
        torch.cuda.empty_cache()
        return h, dt

    def vectors(m):
        g = torch.Generator(device="cuda")
        g.manual_seed(1234)
        return torch.randn((m, 2, N), generator=g, device="cuda", dtype=torch.float64)

    def timed_parts(h, Xv, out, reduced, warmup, steps):
        for s_ in range(warmup):
            h.sigma_part(Xv, out, s_ % PRODUCT_PARTS, PRODUCT_PARTS, reduced=reduced)
        torch.cuda.synchronize()
        h.reset_stats()
        t0 = time.perf_counter()
        for s_ in range(warmup, warmup + steps):
            h.sigma_part(Xv, out, s_ % PRODUCT_PARTS, PRODUCT_PARTS, reduced=reduced)
            log(f"{'reduced' if reduced else 'fp64'} step {s_ - warmup + 1}/{steps} (part {s_ % PRODUCT_PARTS}) "
                f"at {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, h.stats()

    # reduced precision: the headline
    h, setup_red = make_handle(PRECISIONS[prec_name])
    log(f"{prec_name} handle set up in {setup_red:.1f} s ({h.device_bytes() / 2**30:.1f} GiB)")
    Xv = vectors(PRODUCT_M)
    out = torch.empty_like(Xv)
    elapsed, st = timed_parts(h, Xv, out, True, args.warmup, args.steps)
    if not args.no_fp64:
        # one complete reduced pass on a 2N-vector, compared below with the FP64 pass
        X1 = vectors(1)
        red1 = torch.empty_like(X1)
        h.sigma_device(X1, red1, reduced=True)
        red1 = red1.cpu().numpy()
    h.close()
    del Xv, out
    torch.cuda.empty_cache()
    value = st["product_flops"] / elapsed / 1e12
    rows_timed = args.steps * o / PRODUCT_PARTS
    h_n = st["hhat_launches"]
    achieved = st["hhat_flops"] / st["hhat_seconds"] / 1e12 if st["hhat_seconds"] > 0 else 0.0
    flops_per_launch = st["hhat_flops"] / max(h_n, 1)
    # algorithmic bytes of one launch: the split strip [rows v][N] and G [16 naux][N] read once
    # (4 bytes a value), H [16 naux][rows v] written once
    strip_rows_v = PRODUCT_STRIP_ROWS * v
    kX = 2 * PRODUCT_M * X
    hhat_bytes = 4.0 * (strip_rows_v * N + kX * N + strip_rows_v * kX)
    log(f"reduced: {value:.1f} TF/s over {args.steps} steps, amplitude GEMM {achieved:.1f} TF/s")

    rel_total = rel_second = fp64_tflops = fp64_hhat = None
    fsteps = 0
    if not args.no_fp64:
        # FP64 beside it: same step, 4 trial vectors (memory), and the FP64 pass on the reduced one's vectors
        hf, setup64 = make_handle(P.PP_FP64)
        log(f"fp64 handle set up in {setup64:.1f} s")
        Xf = vectors(PRODUCT_M_FP64)
        outf = torch.empty_like(Xf)
        fsteps = max(1, min(2, args.steps))
        elf, stf = timed_parts(hf, Xf, outf, False, 1 if args.warmup else 0, fsteps)
        ref1 = torch.empty_like(X1)
        hf.sigma_device(X1, ref1)
        first1 = torch.empty_like(X1)
        hf.sigma_device(X1, first1, order=1)
        ref1, first1 = ref1.cpu().numpy(), first1.cpu().numpy()
        hf.close()
        del Xf, outf
        torch.cuda.empty_cache()
        err = np.abs(red1 - ref1).max()
        rel_total = float(err / np.abs(ref1).max())
        rel_second = float(err / np.abs(ref1 - first1).max())
        fp64_tflops = stf["product_flops"] / elf / 1e12
        fp64_hhat = stf["hhat_flops"] / stf["hhat_seconds"] / 1e12 if stf["hhat_seconds"] > 0 else 0.0
        log(f"fp64: {fp64_tflops:.1f} TF/s, amplitude GEMM {fp64_hhat:.1f} TF/s; reduced vs FP64 rel err "
            f"{rel_total:.2e} (second-order part {rel_second:.2e})")

    line = {
        "metric": "window solves/sec + sigma-build TFLOP/s at 1e-6 Ha; p50/p99 solve latency",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[prec_name],
        "data": "synthetic (seeded device generator; PbS/CdS orbitals and integrals are not available)",
        "config": {"workload": f"{PRODUCT_WORKLOAD}: second-order product pass M X, n_occ={o}, n_vir={v}, "
                               f"n_aux={X}, {PRODUCT_M} trial 2N-vectors ({2 * PRODUCT_M} particle-hole vectors), "
                               f"amplitudes rebuilt in strips of {PRODUCT_STRIP_ROWS} occupied rows, issued as "
                               f"{PRODUCT_PARTS} parts of {o // PRODUCT_PARTS} rows; one step = one part",
                   "parts_per_pass": PRODUCT_PARTS, "strip_rows": PRODUCT_STRIP_ROWS, "vectors": 2 * PRODUCT_M,
                   "precision": f"{prec_name} contractions (split-BF16 amplitude products, FP32 elsewhere), "
                                f"FP64 diagonal terms and assembly",
                   "parallelism": "single GPU"},
        "sigma_tflops": value,
        "setup_seconds": setup_red,
        "reduced_vs_fp64_max_rel_error": rel_total,
        "reduced_vs_fp64_rel_error_of_second_order_part": rel_second,
        "fp64_sigma_tflops": fp64_tflops,
        "fp64_amplitude_gemm_tflops": fp64_hhat,
        "fp64_vectors": 2 * PRODUCT_M_FP64,
        "fp64_steps": fsteps,
        "reduced_over_fp64": value / fp64_tflops if fp64_tflops else None,
        "roofline": {"bound": "mfma",
                     "kernel": "gemm_sbf16_kernel<256,256,4,2,2,1> (H = tau G of one amplitude strip: split-BF16, "
                               "three BF16 MFMAs per FP32-equivalent product), priced against the BF16 peak / 3",
                     "achieved": achieved, "peak": PEAK_SPLIT_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_SPLIT_BF16_TFLOPS,
                     "launches": h_n, "avg_launch_ms": 1e3 * st["hhat_seconds"] / max(h_n, 1),
                     "flops_per_launch": flops_per_launch,
                     "traffic": product_traffic(flops_per_launch),
                     "algorithmic_bytes_per_launch": hhat_bytes},
    }
    # the 40/160/600 window solves beside it (FP64 and the reduced precision)
    if not args.no_windows:
        wargs = argparse.Namespace(**vars(args))
        wargs.copy_calibration = False
        wargs.windows = 0
        for pn in ("fp64", prec_name):
            w = windows_run(wargs, "mp2_o40_v160_x600", pn, 2, 1, False)
            line[f"windows_mp2_o40_v160_x600_{pn}"] = {
                key: w[key] for key in ("value", "unit", "windows_meeting_tolerance", "max_abs_dE_ha", "max_rel_df",
                                         "latency_p50_s", "latency_p99_s", "products_per_window", "sigma_tflops")}
            line[f"windows_mp2_o40_v160_x600_{pn}"]["amplitude_gemm_tflops"] = w["roofline"]["achieved"]
            log(f"windows {pn}: {w['value']:.2f} solves/s ({w['windows_meeting_tolerance']})")
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = product_cpu_baseline(o, v, X, seed, 2 * PRODUCT_M, st["product_flops"] / (rows_timed * v))
    print(json.dumps(line), flush=True)

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described but not implemented)"}))
        sys.exit(2)
    if args.riesz:
        riesz_main(args)
        return
    if args.serve:
        serve_main(args)
        return
    if args.large:
        large_main(args)
        return
    if args.workload != PRODUCT_WORKLOAD:
        line = windows_run(args, args.workload, args.precision or "fp64", args.steps, args.warmup,
                           not args.no_cpu_baseline)
        print(json.dumps(line), flush=True)
        return
    product_main(args)


if __name__ == "__main__":
    main()
