"""Solver service: Poisson-arriving requests (implicit time steps of a warm
bubble on one of several grids and degrees) served with continuous batching.

A request is admitted in arrival order as soon as its workspace fits in the
batch arena (the HBM budget) and a member slot is free; from then on the
batch's workers advance it step by step beside every other admitted request,
and it leaves the batch (returning its arena range) when its last step is
done.  Latency is arrival to completion.  The scheduling loop only talks to
an object with the jfmg.Batch methods, so it can be exercised with a
simulated batch on the host.
"""
from __future__ import annotations

import time
from collections import deque


def serve(requests, batch, need_bytes, arena_bytes, clock=time.perf_counter, sleep=time.sleep,
          time_scale=1.0, keep_state=False):
    """Serve `requests` (dicts with id, arrival [s], cfg, pert, steps) on `batch`.

    need_bytes(cfg) is a request's workspace size; requests larger than the
    whole arena are rejected at arrival (status "rejected").  Arrival times are
    multiplied by time_scale.  Returns one record per request, in id order."""
    pending = deque(sorted(requests, key=lambda r: (r["arrival"], r["id"])))
    queue = deque()
    active = {}
    records = {}
    t0 = clock()
    batch.start()
    try:
        while pending or queue or active:
            now = clock() - t0
            while pending and pending[0]["arrival"] * time_scale <= now:
                r = pending.popleft()
                rec = {"id": r["id"], "arrival": r["arrival"] * time_scale, "steps": r["steps"],
                       "ndof": 4 * r["cfg"]["nx"] * r["cfg"]["nz"] * (r["cfg"]["k"] + 1) ** 2}
                records[r["id"]] = rec
                if need_bytes(r["cfg"]) > arena_bytes:
                    rec.update(status="rejected", completed=now, latency=now - rec["arrival"])
                else:
                    queue.append(r)
            # first come, first served: the head waits until it fits
            while queue:
                r = queue[0]
                slot = batch.admit(r["cfg"], r["steps"], r["pert"])
                if slot is None:
                    break
                queue.popleft()
                records[r["id"]]["admitted"] = clock() - t0
                active[slot] = r["id"]
            next_arrival = pending[0]["arrival"] * time_scale - (clock() - t0) if pending else None
            if not active:
                if next_arrival is not None:
                    sleep(max(next_arrival, 0.0))
                elif queue:   # nothing runs and the head does not fit: cannot happen after the size check
                    raise RuntimeError("request does not fit an empty arena")
                continue
            timeout = max(next_arrival, 1e-4) if next_arrival is not None else 1.0
            slot = batch.wait_any(timeout)
            if slot is None:
                continue
            done_at = clock() - t0
            finished, steps_done, stats = batch.poll(slot)
            U = batch.retire(slot)
            rid = active.pop(slot)
            rec = records[rid]
            rec.update(completed=done_at, latency=done_at - rec["arrival"], steps_done=steps_done,
                       status="ok" if stats["status"] == 0 else f"error {stats['status']}",
                       newton_its=stats["newton_its"], gmres_its=stats["gmres_its"],
                       stall_stops=stats.get("stall_stops", 0), reorth_its=stats.get("reorth_its", 0),
                       reached_rtol=stats.get("reached_rtol", 0.0))
            if keep_state:
                rec["U"] = U
    finally:
        batch.stop()
    return [records[i] for i in sorted(records)]


def summary(records):
    """Throughput (DOF-Newton-steps/s over the makespan) and latency percentiles."""
    ok = [r for r in records if r.get("status") == "ok"]
    if not ok:
        return {"requests": len(records), "completed": 0}
    t_first = min(r["arrival"] for r in records)
    t_last = max(r["completed"] for r in ok)
    work = sum(r["ndof"] * r["steps"] for r in ok)
    lat = sorted(r["latency"] for r in ok)

    def pct(q):
        return lat[min(len(lat) - 1, max(0, int(round(q / 100.0 * (len(lat) - 1)))))]

    return {"requests": len(records), "completed": len(ok),
            "rejected": sum(1 for r in records if r.get("status") == "rejected"),
            "makespan_s": t_last - t_first, "dof_newton_steps": work,
            "value": work / (t_last - t_first) if t_last > t_first else None,
            "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99),
            "newton_its": sum(r["newton_its"] for r in ok), "gmres_its": sum(r["gmres_its"] for r in ok)}


def serial_fifo(requests, service_s):
    """Latencies of a one-at-a-time FIFO server with the given service times."""
    t = 0.0
    out = []
    for r, s in sorted(zip(requests, service_s), key=lambda x: (x[0]["arrival"], x[0]["id"])):
        t = max(t, r["arrival"]) + s
        out.append(t - r["arrival"])
    return out
