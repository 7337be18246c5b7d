"""Benchmark: DOF-Newton-steps/s of the implicit DG solver on one MI355X.

A step is one implicit SDIRK2 step of the density-current workload (256 x 64
quads, k = 3, viscous, dt = 2 s, Newton rtol 1e-8, FGMRES(30), 4 FV levels,
mg002222V, one-stage RK smoother) with the whole solver on the GPU: residuals,
FD Jacobian-vector products, transfers, FV multigrid and Arnoldi.  value =
(timed steps x unknowns) / wall seconds, inputs resident in HBM.  The plain
FP64 form is the headline; the FP32-multigrid form is timed beside it.

Prints ONE JSON line.  --gpus > 1 is not supported (the solver runs on one GPU).
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

# HBM bytes per launch of the FV smoother-stage kernel class fv_stage (the
# wide-tile kernel: levels of 1024x256 and 512x128 cells), from two
# rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE) over
#   bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp32 --no-forms --profile-class fv_stage
# averaged over its launches, each counter scaled by what it reads for the 1 GiB
# device copy of that same run (FETCH_SIZE x2, WRITE_SIZE x1).
# It describes the kernel sources hashed below and is reported as null once
# they change.
TRAFFIC = {"class": "fv_stage", "bytes_per_launch": 2.9739e+07,
           "sources": ["paper_2505_24504_amd/csrc/fv.hip", "paper_2505_24504_amd/csrc/jfmg_dev.h",
                       "paper_2505_24504_amd/csrc/jfmg_internal.h"],
           "sha256": "1ddb92973a0fc83dc3e7d5774a9c48fffa4a6ea16e023bbead5fa1f1b62ccb65",
           "profile": "profiles/traffic_fv_stage_density_current_fp64.md"}


def measured_traffic(cls):
    """Counter-measured HBM bytes per launch of `cls`, if taken on the current kernel sources."""
    import hashlib
    if cls != TRAFFIC["class"]:
        return None
    h = hashlib.sha256()
    for s in TRAFFIC["sources"]:
        with open(os.path.join(ROOT, s), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC["bytes_per_launch"] if h.hexdigest() == TRAFFIC["sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the ensemble, serving and inertia-gravity forms")
    ap.add_argument("--serve-requests", type=int, default=500,
                    help="requests of the seed-5 stream served at saturation (FP32 and FP64 multigrid)")
    ap.add_argument("--serve-sweep-requests", type=int, default=200,
                    help="requests per offered rate below saturation")
    ap.add_argument("--serial-requests", type=int, default=100,
                    help="requests of the stream solved one at a time with the FP64 multigrid")
    ap.add_argument("--cpu-repeats", type=int, default=3,
                    help="oracle runs of the headline step (median; fewer if one takes over a minute)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the HBM-resident (above cache size) kernel measurements")
    ap.add_argument("--profile-class", default="auto",
                    help="kernel class timed with HIP events ('auto': largest total time)")
    return ap.parse_args()


def progress(msg):
    """One line per finished part of the benchmark on stderr (the JSON line stays on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def run_form(d, pert, steps, warmup, profile_classes, tune=False):
    """Warm-up and timed implicit steps, with the library's default FV tile shapes
    (the same in every pass and under the profilers) or, with tune, the shapes the
    autotuner picks at the initial state (setup, outside the timed region)."""
    import torch

    from paper_2505_24504_amd import jfmg
    p = jfmg.Problem(d, device="cuda:0")
    U = p.initial_state(pert)
    if tune:
        p.linearize(U, (1.0 - 2.0 ** -0.5) * d["dt"])
        p.autotune(reps=20)
    p.tiles = p.get_tiles()
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


def autotune_report(d, pert):
    """What the autotuner chooses for the workload at its initial state (FP64 and
    FP32 multigrid): the mean stage-kernel time of every tile shape per level."""
    from paper_2505_24504_amd import jfmg
    out = {}
    for prec in (64, 32):
        p = jfmg.Problem(dict(d, mg_precision=prec), device="cuda:0")
        U = p.initial_state(pert)
        p.linearize(U, (1.0 - 2.0 ** -0.5) * d["dt"])
        default = p.get_tiles()
        choice, times = p.autotune(reps=20)
        out[f"fp{prec}"] = {"default": default, "choice": choice,
                            "stage_us": {str(l): {s: round(t, 2) for s, t in v.items()} for l, v in times.items()}}
        del p
    return out


def stream_copy(nbytes, reps=20, triad=False):
    """STREAM-style device copy y = x (2 arrays moved) or triad z = x + s y (3 arrays)
    over nbytes per array: GB/s of the arrays moved."""
    import torch
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    z = torch.empty_like(x) if triad else None
    y.fill_(2.0)

    def once():
        if triad:
            torch.add(x, y, alpha=3.0, out=z)
        else:
            y.copy_(x)
    once()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y, z
    return (3.0 if triad else 2.0) * n * 8 / (ms * 1e-3) / 1e9


def _sync():
    import torch
    torch.cuda.synchronize()


def _lockstep_ensemble(mem, prec):
    """The members of each grid size form one lock-step problem (every kernel launch
    covers all of them, tiles by the autotuner); the three problems run concurrently."""
    import torch
    from paper_2505_24504_amd import jfmg
    groups = {}
    for d, pert, n in mem:
        groups.setdefault((d["nx"], d["nz"]), []).append((dict(d, mg_precision=prec), pert, n))
    b = jfmg.Batch(48 << 30, max_members=len(groups), workers=len(groups), device="cuda:0")
    gslots = []
    for ms in groups.values():
        single = jfmg.Problem(ms[0][0], device="cuda:0")
        U = torch.cat([single.initial_state(pert) for _, pert, _ in ms])
        del single
        gslots.append(b.admit(dict(ms[0][0], batch=len(ms)), ms[0][2], None, U))
    t0 = time.perf_counter()
    tiles = [b.autotune(s_) for s_ in gslots]
    el_tune = time.perf_counter() - t0
    _sync()
    t0 = time.perf_counter()
    b.run()
    el = time.perf_counter() - t0
    polled = [b.poll(s_) for s_ in gslots]
    b.close()
    ok = sum(len(ms) for ms, (f_, _, st) in zip(groups.values(), polled) if f_ and st["status"] == 0)
    return el, {"members_ok": ok, "groups": [len(ms) for ms in groups.values()], "tiles": tiles,
                "autotune_seconds": el_tune, "lockstep_gmres_its": [st["gmres_its"] for _, _, st in polled],
                "stall_stops": sum(st["stall_stops"] for _, _, st in polled),
                "reorth_its": sum(st["reorth_its"] for _, _, st in polled),
                "reached_rtol": max(st["reached_rtol"] for _, _, st in polled)}


def _ragged_ensemble(mem, prec, graphs=False):
    """All members in one ragged batch (one problem; every kernel one launch over the 64
    members of three grid sizes, tiles by the autotuner on the batch), 5 steps; with
    graphs, every FGMRES iteration replays a captured HIP graph."""
    import torch
    from paper_2505_24504_amd import jfmg
    ds = [dict(d, mg_precision=prec) for d, _, _ in mem]
    old = os.environ.get("JFMG_GRAPH")
    os.environ["JFMG_GRAPH"] = "1" if graphs else "0"
    try:
        pb = jfmg.Problem(ds, device="cuda:0")
    finally:
        if old is None:
            del os.environ["JFMG_GRAPH"]
        else:
            os.environ["JFMG_GRAPH"] = old
    U = torch.cat([jfmg.Problem(d, device="cuda:0").initial_state(pert) for d, (_, pert, _) in zip(ds, mem)])
    t0 = time.perf_counter()
    pb.linearize(U, (1.0 - 2 ** -0.5) * ds[0]["dt"])
    tiles, _ = pb.autotune(reps=5)
    el_tune = time.perf_counter() - t0
    steps = mem[0][2]
    its, stalls, reorth, reach, ok = 0, 0, 0, 0.0, True
    _sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = pb.implicit_step(U, raise_on_error=False)
        its += st["gmres_its"]
        stalls += st["stall_stops"]
        reorth += st["reorth_its"]
        reach = max(reach, st["reached_rtol"])
        ok = ok and st["status"] == 0
    _sync()
    el = time.perf_counter() - t0
    return el, {"members_ok": len(mem) if ok else 0, "tiles": tiles, "autotune_seconds": el_tune,
                "lockstep_gmres_its": its, "stall_stops": stalls, "reorth_its": reorth, "reached_rtol": reach, "graphs": graphs,
                "launches": "one per kernel over all 64 members (ragged batch)"}


def ensemble_forms():
    """64-member ensemble (k = 2 warm bubbles on 32x16 / 64x32 / 96x48, 5 SDIRK2 steps
    each): lock-step groups (one batched problem per grid size) with the FP32 and with the
    FP64 multigrid, concurrent single problems from one arena (FP32), and the members run
    one after another (FP64).  Stages may end at the rounding floor of G (stall stops,
    newton_stall 1e-7); reached_rtol is the largest final ||G|| / ||G^0|| of any stage."""
    from paper_2505_24504_amd import jfmg, workloads as W
    mem = W.ensemble(seed=4, members=64)
    work = sum(jfmg.num_dofs(d) * n for d, _, n in mem)
    b = jfmg.Batch(48 << 30, max_members=len(mem), workers=8, device="cuda:0")
    slots = [b.admit(d, n, pert) for d, pert, n in mem]
    _sync()
    t0 = time.perf_counter()
    b.run()
    el_b = time.perf_counter() - t0
    polled = [b.poll(s_) for s_ in slots]
    b.close()
    ok_b = sum(1 for f, _, st in polled if f and st["status"] == 0)
    el_s, its_s, ok_s, stalls_s, reorth_s, reach_s = 0.0, 0, 0, 0, 0, 0.0
    for d, pert, n in mem:
        p = jfmg.Problem(dict(d, mg_precision=64), device="cuda:0")
        U = p.initial_state(pert)
        _sync()
        t0 = time.perf_counter()
        good = True
        for _ in range(n):
            st = p.implicit_step(U, raise_on_error=False)
            its_s += st["gmres_its"]
            stalls_s += st["stall_stops"]
            reorth_s += st["reorth_its"]
            reach_s = max(reach_s, st["reached_rtol"])
            good = good and st["status"] == 0
        _sync()
        el_s += time.perf_counter() - t0
        ok_s += good
        del p
    out = {}
    progress(f"ensemble concurrent and serial forms done ({el_b:.1f} s, {el_s:.1f} s)")
    assert len({n for _, _, n in mem}) == 1
    for prec, graphs in ((32, False), (64, False), (32, True)):
        el_r, info = _ragged_ensemble(mem, prec, graphs)
        key = f"ensemble_ragged_fp{prec}" + ("_graph" if graphs else "")
        out[key] = dict({"value": work / el_r, "seconds": el_r}, **info)
        progress(f"ensemble ragged batch FP{prec}{' graphs' if graphs else ''}: {work / el_r:.3e} DOF-Newton-steps/s")
    for prec in (32, 64):
        el_l, info = _lockstep_ensemble(mem, prec)
        out[f"ensemble_lockstep_fp{prec}"] = dict({"value": work / el_l, "seconds": el_l}, **info)
        progress(f"ensemble lock-step FP{prec}: {work / el_l:.3e} DOF-Newton-steps/s")
    out.update({
        "ensemble_batched_fp32": {"value": work / el_b, "seconds": el_b, "members_ok": ok_b,
                                  "gmres_its": sum(st["gmres_its"] for _, _, st in polled),
                                  "stall_stops": sum(st["stall_stops"] for _, _, st in polled),
                                  "reorth_its": sum(st["reorth_its"] for _, _, st in polled),
                                  "reached_rtol": max(st["reached_rtol"] for _, _, st in polled)},
        "ensemble_serial_fp64": {"value": work / el_s, "seconds": el_s, "members_ok": ok_s,
                                 "gmres_its": its_s, "stall_stops": stalls_s, "reorth_its": reorth_s,
                                 "reached_rtol": reach_s},
        "ensemble_workload": "64 warm bubbles, k=2, grids 32x16/64x32/96x48, 5 SDIRK2 steps each, "
                             f"{work} DOF-Newton-steps; 640 stages"})
    return out


def _serve_once(reqs, prec, rate_scale=1.0):
    """Serve reqs (arrival times scaled by rate_scale) with continuous batching from a
    64 GB arena; returns the summary with the stall statistics."""
    from paper_2505_24504_amd import jfmg, serve
    rq = [dict(r, cfg=dict(r["cfg"], mg_precision=prec)) for r in reqs]
    arena = 64 << 30
    b = jfmg.Batch(arena, max_members=64, workers=8, device="cuda:0")
    recs = serve.serve(rq, b, jfmg.workspace_bytes, arena, time_scale=rate_scale)
    b.close()
    s = serve.summary(recs)
    s["offered_req_per_s"] = len(rq) / (rq[-1]["arrival"] * rate_scale) if rq else None
    s["stall_stops"] = sum(r.get("stall_stops", 0) for r in recs)
    s["reorth_its"] = sum(r.get("reorth_its", 0) for r in recs)
    s["reached_rtol"] = max((r.get("reached_rtol", 0.0) for r in recs), default=0.0)
    return s


def serving_forms(n_sat, n_sweep, n_serial):
    """The seed-5 request stream (Poisson, 200 req/s as configured; grid, k, physics and
    steps drawn per request).  (1) Saturation: the first n_sat requests at the configured
    rate, far above what one GPU sustains, served with continuous batching with the FP32
    and with the FP64 multigrid (throughput = saturation throughput; latency = queueing).
    (2) Load sweep: the first n_sweep requests with arrival times stretched so that the
    offered rate is 0.5 and 0.8 of the FP32 saturation rate (p50/p99 against offered rate).
    (3) The first n_serial requests solved one at a time with the plain FP64 multigrid."""
    from paper_2505_24504_amd import jfmg, serve, workloads as W
    reqs = W.serving_requests(seed=5, n_requests=max(n_sat, n_sweep, n_serial))
    out = {}
    sat = reqs[:n_sat]
    work = sum(jfmg.num_dofs(r["cfg"]) * r["steps"] for r in sat)
    for prec in (32, 64):
        out[f"served_fp{prec}_saturation"] = _serve_once(sat, prec)
        progress(f"served {n_sat} requests at saturation, FP{prec} multigrid: "
                 f"{out[f'served_fp{prec}_saturation']['value']:.3e} DOF-Newton-steps/s")
    # requests per second the FP32 server completes at saturation
    s32 = out["served_fp32_saturation"]
    sat_rate = s32["completed"] / s32["makespan_s"]
    sweep = reqs[:n_sweep]
    base_rate = len(sweep) / sweep[-1]["arrival"]
    out["served_fp32_load_sweep"] = {}
    for frac in (0.5, 0.8):
        scale = base_rate / (frac * sat_rate)
        r = _serve_once(sweep, 32, rate_scale=scale)
        r["fraction_of_saturation"] = frac
        out["served_fp32_load_sweep"][str(frac)] = r
        progress(f"served at {frac} of saturation: p50 {r['p50_ms']:.0f} ms p99 {r['p99_ms']:.0f} ms")
    svc, ok = [], 0
    ser = reqs[:n_serial]
    for r in ser:
        _sync()
        t0 = time.perf_counter()
        p = jfmg.Problem(dict(r["cfg"], mg_precision=64), device="cuda:0")
        U = p.initial_state(r["pert"])
        good = True
        for _ in range(r["steps"]):
            good = good and p.implicit_step(U, raise_on_error=False)["status"] == 0
        _sync()
        svc.append(time.perf_counter() - t0)
        ok += good
        del p
    lat = serve.serial_fifo(ser, svc)
    wser = sum(jfmg.num_dofs(r["cfg"]) * r["steps"] for r in ser)
    out["serial_fp64"] = {"value": wser / sum(svc), "seconds": sum(svc), "completed": ok, "requests": len(ser),
                          "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
                          "note": "latencies of a one-at-a-time FIFO server on the configured arrivals"}
    progress(f"serial FP64 requests done ({sum(svc):.1f} s)")
    out["saturation_req_per_s_fp32"] = sat_rate
    out["serving_workload"] = (f"seed-5 stream (Poisson 200/s), grids 16x8..256x128, k 1..3, Euler or viscous, "
                               f"1..10 SDIRK2 steps; saturation runs: first {n_sat} requests, {work} DOF-Newton-steps; "
                               f"load sweep: first {n_sweep}; serial: first {n_serial}")
    return out


def inertia_gravity_forms(steps=20):
    """Inertia-gravity wave (600x20, k=3, periodic, N = 0.01, 20 m/s wind, dt = 12 s), the
    configured 20 steps: FP32 multigrid against FP64 multigrid, and how far the two solutions
    are apart after the 20 steps."""
    import numpy as np
    from paper_2505_24504_amd import jfmg, workloads as W
    out, Us = {}, {}
    for prec in (64, 32):
        d, pert, _ = W.inertia_gravity(mg_precision=prec)
        p = jfmg.Problem(d, device="cuda:0")
        U = p.initial_state(pert)
        U0 = U.clone()
        p.implicit_step(U)          # warm-up step, from the same start
        U.copy_(U0)
        _sync()
        t0 = time.perf_counter()
        lat, its = [], []
        for _ in range(steps):
            ts = time.perf_counter()
            its.append(p.implicit_step(U, raise_on_error=False))
            lat.append(time.perf_counter() - ts)
        _sync()
        el = time.perf_counter() - t0
        n = jfmg.num_dofs(d)
        out[f"fp{prec}_mg"] = {"value": steps * n / el, "ms_per_step": 1e3 * el / steps,
                               "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
                               "newton_its": sum(s["newton_its"] for s in its),
                               "gmres_its": sum(s["gmres_its"] for s in its),
                               "stall_stops": sum(s["stall_stops"] for s in its),
                               "reorth_its": sum(s["reorth_its"] for s in its),
                               "reached_rtol": max(s["reached_rtol"] for s in its),
                               "ok": all(s["status"] == 0 for s in its)}
        Us[prec] = (U0.cpu().numpy(), U.cpu().numpy())
        progress(f"inertia-gravity FP{prec} multigrid: {1e3 * el / steps:.1f} ms/step")
        del p
    (a0, a), (_, b) = Us[64], Us[32]
    n4 = a.size // 4
    out["fp32_vs_fp64_rel_l2_of_change"] = [
        float(np.linalg.norm((b - a)[c * n4:(c + 1) * n4]) / max(np.linalg.norm((a - a0)[c * n4:(c + 1) * n4]), 1e-300))
        for c in range(4)]
    out["workload"] = f"inertia-gravity wave, 600x20 quads, k=3, {steps} SDIRK2 steps of 12 s"
    return out


def bubble_small_form(steps=20):
    """The tiny warm bubble (16x16 quads, k = 1, one implicit-Euler step of 1 s, FGMRES(20),
    3 levels, mg002222V with the three-stage smoother), launch-latency bound: time per step
    and per FGMRES iteration at the configured Newton rtol 1e-6 and at 1e-8."""
    from paper_2505_24504_amd import jfmg, workloads as W
    d0, pert, _ = W.bubble_small()
    out = {}
    for rtol in (1e-6, 1e-8):
        d = dict(d0, newton_rtol=rtol)
        p = jfmg.Problem(d, device="cuda:0")
        U0 = p.initial_state(pert)
        U = U0.clone()
        p.implicit_step(U)
        _sync()
        lat, its = [], []
        for _ in range(steps):
            U.copy_(U0)
            _sync()
            ts = time.perf_counter()
            its.append(p.implicit_step(U))
            lat.append(time.perf_counter() - ts)
        g = sum(s["gmres_its"] for s in its)
        out[f"rtol_{rtol:.0e}"] = {"ms_per_step": 1e3 * sum(lat) / steps, "p50_ms": 1e3 * percentile(lat, 50),
                                  "p99_ms": 1e3 * percentile(lat, 99), "gmres_its_per_step": g / steps,
                                  "newton_its_per_step": sum(s["newton_its"] for s in its) / steps,
                                  "us_per_gmres_iteration": 1e6 * sum(lat) / g,
                                  "value": jfmg.num_dofs(d) * steps / sum(lat)}
        del p
    out["workload"] = "warm bubble 16x16 quads, k=1, implicit Euler dt=1 s, FGMRES(20), 3 levels, 3-stage smoother"
    return out


def explicit_reference_form(d, pert, implicit_ms_per_step, reps=5):
    """The paper's reference method beside the implicit solver on the same workload:
    SSP RK(4,3) at dt = h / ((2k+1) 380 m/s), the largest of the tried CFL factors
    that stays finite over 20 s of the density current (1.25x diverges), run over one
    implicit step interval; the SDIRK2 step's relative L2 distance from it at that time
    is the implicit step's time-discretisation error against the reference."""
    import numpy as np
    import torch
    from paper_2505_24504_amd import jfmg
    T = d["dt"]
    h = min((d["x1"] - d["x0"]) / d["nx"], (d["z1"] - d["z0"]) / d["nz"])
    n = int(np.ceil(T / (h / ((2 * d["k"] + 1) * 380.0))))
    dt = T / n
    p = jfmg.Problem(d, device="cuda:0")
    U0 = p.initial_state(pert)
    Ue = U0.clone()
    p.explicit_steps(Ue, dt, n)      # warm-up run, also the reference state at time T
    Ui = U0.clone()
    st = p.implicit_step(Ui)
    U = U0.clone()
    _sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        p.explicit_steps(U, dt, n)
    _sync()
    el = (time.perf_counter() - t0) / reps
    N = jfmg.num_dofs(d)
    # the implicit step's cost per simulated second at larger time steps (one warm-up
    # and two timed steps each from the initial state)
    sweep = {}
    for dti in (5.0, 10.0, 20.0):
        q = jfmg.Problem(dict(d, dt=dti), device="cuda:0")
        V = q.initial_state(pert)
        q.implicit_step(V, raise_on_error=False)
        _sync()
        t1 = time.perf_counter()
        sts = [q.implicit_step(V, raise_on_error=False) for _ in range(2)]
        _sync()
        e1 = (time.perf_counter() - t1) / 2
        sweep[str(dti)] = {"ms_per_simulated_s": 1e3 * e1 / dti, "ms_per_step": 1e3 * e1,
                           "gmres_its_per_step": sum(x["gmres_its"] for x in sts) / 2,
                           "ok": all(x["status"] == 0 for x in sts)}
        del q, V
    return {"implicit_dt_sweep": sweep, "dt": dt, "steps_per_interval": n, "interval_s": T,
            "explicit_ms_per_simulated_s": 1e3 * el / T,
            "implicit_ms_per_simulated_s": implicit_ms_per_step / T,
            "explicit_dof_steps_per_s": n * N / el,
            "dg_stage_us": 1e6 * el / (4 * n),
            "implicit_vs_explicit_rel_l2": float((Ui - Ue).norm() / (Ue - U0).norm()),
            "implicit_newton_its": st["newton_its"], "implicit_gmres_its": st["gmres_its"],
            "finite": bool(torch.isfinite(U).all().item())}


def preconditioner_keys(steps=2):
    """The paper's preconditioner configurations (key mg a b c d e f G) on the three
    workload shapes of its experiments: time, FGMRES iterations and operator calls per
    implicit step (one warm-up step, then `steps` timed ones, FP64 multigrid, one-stage
    smoother; DG-level smoothing at c*_DG = 0.3)."""
    import torch
    from paper_2505_24504_amd import jfmg, workloads as W
    dc, dc_pert, _ = W.density_current()
    ig, ig_pert, _ = W.inertia_gravity(mg_precision=64)
    rb, rb_pert, _ = W.bubble_small()
    rb = dict(rb, nx=64, nz=64, k=2, scheme=1, mg_levels=4, rk_stages=1, newton_rtol=1e-8, gmres_m=30)
    cases = {"density_current_256x64_k3": (dc, dc_pert), "inertia_gravity_600x20_k3": (ig, ig_pert),
             "rising_bubble_64x64_k2": (rb, rb_pert)}
    out = {}
    for wname, (d0, pert) in cases.items():
        res = {}
        for key in ("mg002222V", "mg001111V", "mg111111V", "mg001111W", "mg111111W"):
            d = dict(d0, mg_key=key, pseudo_cfl_dg=0.3, mg_precision=64)
            p = jfmg.Problem(d, device="cuda:0")
            U = p.initial_state(pert)
            st0 = p.implicit_step(U, raise_on_error=False)
            _sync()
            t0 = time.perf_counter()
            sts = [p.implicit_step(U, raise_on_error=False) for _ in range(steps)]
            _sync()
            el = (time.perf_counter() - t0) / steps
            res[key] = {"ms_per_step": 1e3 * el,
                        "gmres_its_per_step": sum(x["gmres_its"] for x in sts) / steps,
                        "jvps_per_step": sum(x["jvps"] for x in sts) / steps,
                        "fv_matvecs_per_step": sum(sum(x["fv_matvecs"]) for x in sts) / steps,
                        "ok": st0["status"] == 0 and all(x["status"] == 0 for x in sts)}
            del p, U
        out[wname] = res
        progress(f"preconditioner keys on {wname} done")
    return out


def large_roofline(reps=20):
    """The FV operator and the DG JVP on vectors far above the 256 MB cache:
    a 1024x1024-quad, k = 3 problem (FV level 4096x4096 cells, DG vector 537 MB,
    density-current physics).  GB/s of algorithmic bytes of the whole call: an FV
    matvec call reads x for ||x|| (eps), then u, F0 and x (with halo) and writes
    g'x (5 vectors); a JVP call reads y for ||y||, then U and y, and writes the
    product (4 vectors).  Events on the launch stream bracket `reps` back-to-back
    calls."""
    import ctypes
    import torch
    from paper_2505_24504_amd import jfmg, workloads as W
    out = {}
    d0, pert, _ = W.density_current()
    for prec in (64, 32):
        # 25.6 km high: the isentropic background stays physical (T > 0) up to ~30 km
        d = dict(d0, nx=1024, nz=1024, z1=25600.0, gmres_m=2, mg_precision=prec)
        p = jfmg.Problem(d, device="cuda:0")
        U = p.initial_state(pert)
        p.linearize(U, 0.5)
        nfv = p.fv_size(0)
        g = torch.Generator(device="cuda:0").manual_seed(7)
        x = torch.randn(nfv, generator=g, device="cuda:0", dtype=p.fv_dtype)
        y = torch.randn(p.ndof, generator=g, device="cuda:0", dtype=torch.float64)
        xo = torch.empty_like(x)
        yo = torch.empty_like(y)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr())
        res = {}
        for name, call, nbytes in (
                ("fv_matvec_4096x4096", lambda: p.L.jfmg_fv_matvec(p.h, 0, ptr(x), ptr(xo)), 5 * nfv * x.element_size()),
                # ||y||^2 pass, then U', y in, G'y out, and the linearization state's volume
                # fluxes and face terms (8 + 8 doubles per node at k = 3)
                ("dg_jvp_1024x1024_k3", lambda: p.L.jfmg_jvp(p.h, ptr(y), ptr(yo)),
                 4 * p.ndof * 8 + 8 * (8 * (p.ndof // 4) + 8 * (p.ndof // 64) * 16))):
            if prec == 32 and name.startswith("dg"):
                continue
            assert call() == 0
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / reps
            gbs = nbytes / (us * 1e-6) / 1e9
            res[name] = {"us": us, "algorithmic_MB": nbytes / 1e6, "GBs": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS}
        out[f"fp{prec}"] = res
        del p, U, x, y, xo, yo
        torch.cuda.empty_cache()
    return out


def host_info():
    """CPU model and core counts of the host the benchmark runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(repeats=3):
    """The oracle timed on the host on the headline workload itself: the first SDIRK2 step
    of the density current (256 x 64 quads, k = 3, 1 048 576 unknowns, same solver
    settings), from the initial state, median of `repeats` runs (one run when the first
    takes over a minute).  The oracle's element and cell loops run on OMP_NUM_THREADS
    threads (default: every usable core); norms and inner products stay serial."""
    h = host_info()
    threads = int(os.environ.get("OMP_NUM_THREADS") or h["usable_cpus"] or 1)
    os.environ["OMP_NUM_THREADS"] = str(threads)   # read when the oracle library loads
    import oracle
    from paper_2505_24504_amd import workloads as W
    d, pert, _ = W.density_current()
    o = oracle.Oracle(d)
    U0 = o.initial_state(pert)
    times, st, rc = [], None, None
    for i in range(repeats):
        t0 = time.perf_counter()
        rc, _, st = o.implicit_step(U0)
        times.append(time.perf_counter() - t0)
        progress(f"oracle step {i + 1}: {times[-1]:.1f} s")
        if times[0] > 60.0:
            break
    el = sorted(times)[len(times) // 2]
    return {"value": o.ndof / el, "unit": "DOF-Newton-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first SDIRK2 step of the density current (256x64 quads, k=3, N={o.ndof}), FP64 C with "
                      f"OpenMP over elements and cells on {threads} threads; median of {len(times)} runs "
                      f"({', '.join(f'{t:.1f}' for t in times)} s); newton {st['newton_its']} gmres "
                      f"{st['gmres_its']}, status {rc}",
            "host": h}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2505_24504_amd import jfmg, workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    jfmg.load_library()
    d, pert, _ = W.density_current()
    N = 4 * d["nx"] * d["nz"] * (d["k"] + 1) ** 2

    # pass 1 (untimed for the metric): find the kernel class with the largest total time
    prof_cls = a.profile_class
    # kernel-class time per FGMRES iteration of one step (event-timed, eager launches), FP64
    # and FP32 multigrid: where an iteration's time goes in either precision
    breakdown = {}
    for prec in (64, 32) if not a.no_fp32 else (64,):
        _, _, _, its_b, prof_b = run_form(dict(d, mg_precision=prec), pert, 1, 0, jfmg.KERNEL_CLASSES)
        g = max(1, sum(st_["gmres_its"] for st_ in its_b))
        breakdown[f"fp{prec}"] = {"gmres_its": g, "us_per_iteration": {
            k: round(1e3 * v["ms"] / g, 2) for k, v in prof_b.items() if v["launches"]},
            "launches_per_iteration": {k: round(v["launches"] / g, 2) for k, v in prof_b.items() if v["launches"]}}
        if prec == 64 and prof_cls == "auto":
            prof_cls = max(prof_b, key=lambda k: prof_b[k]["ms"])
    # timed pass, FP64 multigrid (headline): no instrumentation
    p, el, lat, its, _ = run_form(d, pert, a.steps, a.warmup, [])
    value = a.steps * N / el
    progress(f"headline: {value:.4e} DOF-Newton-steps/s, {1e3 * el / a.steps:.2f} ms/step")
    # second timed pass of the same workload: the dominant kernel class timed by the
    # start/stop events of its own dispatches (eager launches; see include/jfmg.h)
    _, el_prof, _, _, prof = run_form(d, pert, a.steps, a.warmup, [prof_cls])
    pc = prof[prof_cls]
    avg_ms = pc["ms"] / max(pc["launches"], 1)
    bytes_per_launch = pc["bytes"] / max(pc["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if pc["launches"] else None
    forms = {"fp64_mg": {"value": value, "ms_per_step": 1e3 * el / a.steps,
                         "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
                         "tiles": p.tiles}}
    forms["autotune"] = autotune_report(d, pert)
    # other preconditioner configurations of the same workload (same rtol, same steps)
    for name, kw in () if a.no_forms else (("fp64_mg_3stage_smoother", dict(rk_stages=3)),
                     ("fp64_mg111111V_dg_smoothing", dict(mg_key="mg111111V", pseudo_cfl_dg=0.3)),
                     ("fp64_mg112222V_dg_smoothing", dict(mg_key="mg112222V", pseudo_cfl_dg=0.1)),
                     ("fp64_mg_l2_projection_transfer", dict(transfer=1)),
                     ("fp64_mg_interpolation_without_mass_fix", dict(mass_fix=0))):
        try:
            _, elv, latv, itsv, _ = run_form(dict(d, **kw), pert, a.steps, a.warmup, [])
        except Exception as ex:   # a configuration that does not converge is reported, not fatal
            forms[name] = {"config": kw, "error": str(ex)}
            continue
        progress(f"form {name}: {1e3 * elv / a.steps:.1f} ms/step")
        forms[name] = {"value": a.steps * N / elv, "ms_per_step": 1e3 * elv / a.steps, "config": kw,
                       "p50_ms": 1e3 * percentile(latv, 50), "p99_ms": 1e3 * percentile(latv, 99),
                       "newton_its": sum(s["newton_its"] for s in itsv),
                       "gmres_its": sum(s["gmres_its"] for s in itsv), "jvps": sum(s["jvps"] for s in itsv),
                       "reorth_its": sum(s["reorth_its"] for s in itsv),
                       "ok": all(s["status"] == 0 for s in itsv)}
    if not a.no_fp32:
        d32 = dict(d, mg_precision=32)
        p32, el32, lat32, its32, _ = run_form(d32, pert, a.steps, a.warmup, [], tune=True)
        forms["fp32_mg"] = {"value": a.steps * N / el32, "ms_per_step": 1e3 * el32 / a.steps, "tiles": p32.tiles,
                            "p50_ms": 1e3 * percentile(lat32, 50), "p99_ms": 1e3 * percentile(lat32, 99),
                            "newton_its": sum(s["newton_its"] for s in its32),
                            "gmres_its": sum(s["gmres_its"] for s in its32),
                            "reorth_its": sum(s["reorth_its"] for s in its32),
                            "reached_rtol": max(s["reached_rtol"] for s in its32)}
    forms["fp64_mg"]["newton_its"] = sum(s["newton_its"] for s in its)
    forms["fp64_mg"]["gmres_its"] = sum(s["gmres_its"] for s in its)
    forms["fp64_mg"]["reorth_its"] = sum(s["reorth_its"] for s in its)
    forms["fp64_mg"]["reached_rtol"] = max(s["reached_rtol"] for s in its)
    forms["iteration_breakdown"] = breakdown
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
                               "1-stage (explicit Euler) pseudo-time smoother, FP64 multigrid",
                   "unknowns": N, "fd_eps_mode": d["fd_eps_mode"]},
        "p50_ms": 1e3 * percentile(lat, 50),
        "p99_ms": 1e3 * percentile(lat, 99),
        "iterations": {"newton": sum(s["newton_its"] for s in its), "gmres": sum(s["gmres_its"] for s in its),
                       "lh_evals": sum(s["lh_evals"] for s in its), "jvps": sum(s["jvps"] for s in its),
                       "fv_matvecs_per_level": [sum(s["fv_matvecs"][l] for s in its) for l in range(4)],
                       "host_syncs": sum(s["host_syncs"] for s in its),
                       "reorth_its": sum(s["reorth_its"] for s in its)},
        "forms": forms,
        "roofline": {"bound": "hbm", "kernel": prof_cls, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic(prof_cls), "traffic_unit": "bytes per launch",
                     "avg_launch_us": 1e3 * avg_ms, "launches": pc["launches"],
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "timing": "HIP start/stop events of each dispatch of the kernel class, second timed pass "
                               f"of the same {a.steps} steps ({1e3 * el_prof / a.steps:.1f} ms/step with the events)"},
    }
    if not a.no_forms:
        forms["bubble_small"] = bubble_small_form()
        progress("tiny bubble done")
        forms.update(ensemble_forms())
        forms.update(serving_forms(a.serve_requests, a.serve_sweep_requests, a.serial_requests))
        forms["inertia_gravity"] = inertia_gravity_forms()
        forms["explicit_reference"] = explicit_reference_form(d, pert, 1e3 * el / a.steps)
        progress("explicit reference done")
        forms["preconditioner_keys"] = preconditioner_keys()
        progress("preconditioner keys done")
    if not a.no_large:
        out["roofline_hbm_resident"] = large_roofline()
    # copy and triad bandwidth of the device: HBM-resident (1 GiB) and cache-resident (32 MiB)
    hbm_copy, mall_copy = stream_copy(1 << 30), stream_copy(32 << 20)
    hbm_triad, mall_triad = stream_copy(1 << 30, triad=True), stream_copy(32 << 20, triad=True)
    out["stream_copy"] = {"hbm_1GiB_GBs": hbm_copy, "mall_32MiB_GBs": mall_copy,
                          "triad_hbm_1GiB_GBs": hbm_triad, "triad_mall_32MiB_GBs": mall_triad,
                          "roofline_frac_vs_hbm_copy": achieved / hbm_copy if achieved else None,
                          "roofline_frac_vs_mall_copy": achieved / mall_copy if achieved else None}
    out["host"] = host_info()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.cpu_repeats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
