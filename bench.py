"""Benchmark: second-order window solves on one MI355X.

Workload (one "step"): the seeded MP2-corrected system with n_occ = 40,
n_vir = 160, n_aux = 600 (particle-hole dimension 6,400), amplitudes stored,
FP64 throughout.  A step runs the whole hot path on inputs already resident in
HBM: pp_setup (layouts, MP2 densities and ring intermediate from amplitude
strips, Jacobi diagonal), then four window solves at omega0 = 0.3, 0.6, 0.9,
1.2 Ha with 10 roots each (energies, eigenvectors, dipole oscillator
strengths) in one batched call (one solver thread per window, products of
all windows merged into shared passes), then pp_destroy.  Results are checked against stored oracle values
(1e-6 Ha, 1e-5 relative f) and only windows that meet both count.

Prints ONE JSON line (rank 0).  Extra fields: sigma TFLOP/s (all products),
p50/p99 window latency, accuracy, roofline of the dominant kernel (the
amplitude contraction H = tau G, FP64 MFMA) and the CPU oracle baseline.
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
HBM_TBPS = 8.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mp2_o40_v160_x600")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--windows", type=int, default=0, help="use only the first N windows (profiling)")
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is a design "
                                   "note, not implemented)"}))
        sys.exit(2)
    import torch
    import paper_2512_09811_amd as P
    from synth.gen import CONFIGS, WINDOWS, gen_config

    P.lib()
    name = args.workload
    cfg = CONFIGS[name]
    omegas, nr = WINDOWS[name]
    if args.windows:
        omegas = omegas[: args.windows]
    sys_ = gen_config(name)
    dev = torch.device("cuda:0")
    t = {k: torch.tensor(getattr(sys_, k), dtype=torch.float64, device=dev).contiguous()
         for k in ("eps", "B_oo", "B_ov", "B_vv", "dip")}
    torch.cuda.synchronize()
    precision = P.PP_FP32 if args.precision == "fp32" else P.PP_FP64
    golden_path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    golden = json.load(open(golden_path)) if os.path.exists(golden_path) else None

    def step(record):
        h = P.Handle(t["eps"], t["B_oo"], t["B_ov"], t["B_vv"], t["dip"], order=cfg["order"], device_ptrs=True,
                     precision=precision, store_amplitudes=1)
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

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
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
    n_windows = len(omegas) * args.steps
    value = ok / elapsed if golden is not None else n_windows / elapsed
    peak = PEAK_FP32_MFMA_TFLOPS if args.precision == "fp32" else PEAK_FP64_MFMA_TFLOPS
    achieved = (h_flops / h_sec) / 1e12 if h_sec > 0 else 0.0
    line = {
        "metric": "window solves/sec + sigma-build TFLOP/s at 1e-6 Ha; p50/p99 solve latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (seeded generator; PbS/CdS orbitals and integrals are not available)",
        "config": {"workload": f"{name}: second-order, n_occ={cfg['o']}, n_vir={cfg['v']}, n_aux={cfg['naux']}, "
                               f"{len(omegas)} windows x {nr} roots, amplitudes stored",
                   "windows_ha": [float(x) for x in omegas], "n_roots": nr, "parallelism": "single GPU"},
        "windows_meeting_tolerance": f"{ok}/{total}" if golden is not None else "unchecked",
        "max_abs_dE_ha": max_de,
        "max_rel_df": max_df,
        "sigma_tflops": (prod_flops / prod_sec) / 1e12 if prod_sec > 0 else 0.0,
        "sigma_fraction_of_time": prod_sec / elapsed,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "products_per_window": float(np.mean([r[3]["products"] for res, _ in recs for r in res])),
        "roofline": {"bound": "mfma", "kernel": "gemm_kernel<double,128,128,16,1> (H = tau G)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "launches": h_n, "avg_launch_ms": 1e3 * h_sec / max(h_n, 1),
                     "flops_per_launch": h_flops / max(h_n, 1), "traffic": None},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(name)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
