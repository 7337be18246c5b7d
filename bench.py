"""Benchmark: DOF-Newton-steps/s of the implicit DG solver on one MI355X.

A step is one implicit SDIRK2 step of the density-current workload (256 x 64
quads, k = 3, viscous, dt = 2 s, Newton rtol 1e-8, FGMRES(30), 4 FV levels,
mg002222V, 3-stage RK smoother) with the whole solver on the GPU: residuals,
FD Jacobian-vector products, transfers, FV multigrid and Arnoldi.  value =
(timed steps x unknowns) / wall seconds, inputs resident in HBM.  The plain
FP64 form is the headline; the FP32-multigrid form is timed beside it.

Prints ONE JSON line.  --gpus > 1 is not supported (one GPU per process and
this build runs on one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--profile-class", default="auto",
                    help="kernel class timed with HIP events ('auto': largest total time)")
    return ap.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def run_form(d, pert, steps, warmup, profile_classes):
    import torch

    from paper_2505_24504_amd import jfmg
    p = jfmg.Problem(d, device="cuda:0")
    U = p.initial_state(pert)
    for _ in range(warmup):
        p.implicit_step(U)
    p.profile_enable(profile_classes)
    torch.cuda.synchronize()
    lat, its = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        st = p.implicit_step(U)
        lat.append(time.perf_counter() - ts)
        its.append(st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = p.profile_read()
    return p, el, lat, its, prof


def stream_copy(nbytes, reps=20):
    """STREAM-style device copy of nbytes (read + write counted): GB/s."""
    import torch
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * n * 8 / (ms * 1e-3) / 1e9


def cpu_baseline():
    """The oracle timed on the host: first SDIRK2 step of the density current on a
    48 x 12 quad grid of the same domain (k = 3, same physics and solver settings)."""
    import oracle
    from paper_2505_24504_amd import workloads as W
    d, pert, _ = W.density_current()
    d = dict(d, nx=48, nz=12)
    o = oracle.Oracle(d)
    U = o.initial_state(pert)
    t0 = time.perf_counter()
    rc, _, st = o.implicit_step(U)
    el = time.perf_counter() - t0
    return {"value": o.ndof / el, "unit": "DOF-Newton-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one SDIRK2 step of the density current on 48x12 quads (k=3, N={o.ndof}), "
                      f"single-threaded FP64 C, {el:.1f} s, newton {st['newton_its']} gmres {st['gmres_its']}, "
                      f"status {rc}"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2505_24504_amd import jfmg, workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    jfmg.load_library()
    d, pert, _ = W.density_current()
    N = 4 * d["nx"] * d["nz"] * (d["k"] + 1) ** 2

    # pass 1 (untimed for the metric): find the kernel class with the largest total time
    prof_cls = a.profile_class
    if prof_cls == "auto":
        _, _, _, _, prof_all = run_form(d, pert, 1, 0, jfmg.KERNEL_CLASSES)
        prof_cls = max(prof_all, key=lambda k: prof_all[k]["ms"])
    # timed pass, FP64 multigrid (headline): captured HIP graphs, no instrumentation
    p, el, lat, its, _ = run_form(d, pert, a.steps, a.warmup, [])
    value = a.steps * N / el
    # second timed pass of the same workload: the dominant kernel class timed by the
    # start/stop events of its own dispatches (eager launches; see include/jfmg.h)
    _, el_prof, _, _, prof = run_form(d, pert, a.steps, a.warmup, [prof_cls])
    pc = prof[prof_cls]
    avg_ms = pc["ms"] / max(pc["launches"], 1)
    bytes_per_launch = pc["bytes"] / max(pc["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if pc["launches"] else None
    forms = {"fp64_mg": {"value": value, "ms_per_step": 1e3 * el / a.steps,
                         "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99)}}
    if not a.no_fp32:
        d32 = dict(d, mg_precision=32)
        _, el32, lat32, its32, _ = run_form(d32, pert, a.steps, a.warmup, [])
        forms["fp32_mg"] = {"value": a.steps * N / el32, "ms_per_step": 1e3 * el32 / a.steps,
                            "p50_ms": 1e3 * percentile(lat32, 50), "p99_ms": 1e3 * percentile(lat32, 99),
                            "newton_its": sum(s["newton_its"] for s in its32),
                            "gmres_its": sum(s["gmres_its"] for s in its32)}
    out = {
        "metric": "DOF-Newton-steps/s at rtol 1e-8, FP32-MG vs FP64 plain; p50/p99 step latency",
        "value": value,
        "unit": "DOF-Newton-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * el / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "density current: viscous flow with gravity, 256x64 quads on 25.6 km x 6.4 km, "
                               "k=3, SDIRK2 dt=2 s, Newton rtol 1e-8, FGMRES(30), 4 FV levels, mg002222V, "
                               "3-stage RK smoother, FP64 multigrid",
                   "unknowns": N, "fd_eps_mode": d["fd_eps_mode"]},
        "p50_ms": 1e3 * percentile(lat, 50),
        "p99_ms": 1e3 * percentile(lat, 99),
        "iterations": {"newton": sum(s["newton_its"] for s in its), "gmres": sum(s["gmres_its"] for s in its),
                       "lh_evals": sum(s["lh_evals"] for s in its), "jvps": sum(s["jvps"] for s in its),
                       "fv_matvecs_per_level": [sum(s["fv_matvecs"][l] for s in its) for l in range(4)],
                       "host_syncs": sum(s["host_syncs"] for s in its)},
        "forms": forms,
        "roofline": {"bound": "hbm", "kernel": prof_cls, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
                     "avg_launch_us": 1e3 * avg_ms, "launches": pc["launches"],
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "timing": "HIP start/stop events of each dispatch of the kernel class, second timed pass "
                               f"of the same {a.steps} steps without graph replay ({1e3 * el_prof / a.steps:.1f} ms/step)"},
    }
    # copy bandwidth of the device: HBM-resident (1 GiB) and cache-resident (32 MiB)
    hbm_copy, mall_copy = stream_copy(1 << 30), stream_copy(32 << 20)
    out["stream_copy"] = {"hbm_1GiB_GBs": hbm_copy, "mall_32MiB_GBs": mall_copy,
                          "roofline_frac_vs_hbm_copy": achieved / hbm_copy if achieved else None,
                          "roofline_frac_vs_mall_copy": achieved / mall_copy if achieved else None}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
