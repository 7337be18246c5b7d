"""Host logic of the serving loop (no GPU): admission in arrival order under the
arena budget, continuous batching, rejection of requests larger than the arena,
and the latency bookkeeping, driven by a simulated batch on a virtual clock."""
import heapq

import pytest

from paper_2505_24504_amd import serve, workloads as W


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeBatch:
    """Members progress independently; a member's steps take step_s(cfg) each.
    Arena accounting mirrors the library's: a member holds need(cfg) bytes from
    admission to retirement."""

    def __init__(self, clock, arena_bytes, max_members, need, step_s):
        self.clock, self.arena, self.max_members = clock, arena_bytes, max_members
        self.need, self.step_s = need, step_s
        self.used = 0
        self.members = {}
        self.events = []
        self.admit_order = []
        self.peak_used = 0
        self.started = False

    def start(self):
        self.started = True

    def stop(self):
        self.started = False

    def admit(self, cfg, steps, pert):
        assert self.started
        nb = self.need(cfg)
        if self.used + nb > self.arena or len(self.members) >= self.max_members:
            return None
        slot = min(set(range(self.max_members)) - set(self.members))
        self.used += nb
        self.peak_used = max(self.peak_used, self.used)
        done = self.clock() + steps * self.step_s(cfg)
        self.members[slot] = (nb, steps, done)
        heapq.heappush(self.events, (done, slot))
        self.admit_order.append(pert["id"])
        return slot

    def wait_any(self, timeout):
        if not self.events:
            self.clock.sleep(timeout)
            return None
        done, slot = self.events[0]
        if done > self.clock() + timeout:
            self.clock.sleep(timeout)
            return None
        heapq.heappop(self.events)
        self.clock.t = max(self.clock.t, done)
        return slot

    def poll(self, slot):
        nb, steps, _ = self.members[slot]
        return True, steps, {"status": 0, "newton_its": 2 * steps, "gmres_its": 10 * steps}

    def retire(self, slot):
        nb, _, _ = self.members.pop(slot)
        self.used -= nb
        return None


def need(cfg):
    return 4 * cfg["nx"] * cfg["nz"] * (cfg["k"] + 1) ** 2 * 8 * 80


def step_s(cfg):
    return 1e-8 * 4 * cfg["nx"] * cfg["nz"] * (cfg["k"] + 1) ** 2


def requests(n=200):
    reqs = W.serving_requests(seed=5, n_requests=n)
    for r in reqs:
        r["pert"] = dict(r["pert"], id=r["id"])
    return reqs


@pytest.mark.parametrize("arena_gb", [0.5, 2.0, 64.0])
def test_admission_fifo_under_budget(arena_gb):
    clock = VirtualClock()
    arena = int(arena_gb * 2**30)
    reqs = requests()
    b = FakeBatch(clock, arena, 32, need, step_s)
    recs = serve.serve(reqs, b, need, arena, clock=clock, sleep=clock.sleep)
    assert len(recs) == len(reqs)
    admitted = [r["id"] for r in sorted(reqs, key=lambda r: r["arrival"]) if need(r["cfg"]) <= arena]
    assert b.admit_order == admitted           # first come, first served
    assert b.peak_used <= arena                # the HBM budget holds at all times
    for r, q in zip(recs, reqs):
        if need(q["cfg"]) > arena:
            assert r["status"] == "rejected"
            continue
        assert r["status"] == "ok"
        assert r["admitted"] >= r["arrival"] - 1e-12
        assert r["latency"] >= q["steps"] * step_s(q["cfg"]) - 1e-9
        assert r["steps_done"] == q["steps"]
    s = serve.summary(recs)
    assert s["completed"] == sum(1 for q in reqs if need(q["cfg"]) <= arena)
    assert s["p50_ms"] <= s["p99_ms"]


def test_small_arena_forces_queueing():
    clock = VirtualClock()
    reqs = requests(100)
    big = int(64 * 2**30)
    small = int(1.2 * 2**30)
    lat_big = serve.summary(serve.serve(reqs, FakeBatch(clock, big, 64, need, step_s), need, big,
                                        clock=clock, sleep=clock.sleep))
    clock2 = VirtualClock()
    lat_small = serve.summary(serve.serve(reqs, FakeBatch(clock2, small, 64, need, step_s), need, small,
                                          clock=clock2, sleep=clock2.sleep))
    assert lat_small["p99_ms"] > lat_big["p99_ms"]


def test_serial_fifo_latency():
    reqs = [{"id": i, "arrival": a} for i, a in enumerate([0.0, 0.1, 0.2, 5.0])]
    lat = serve.serial_fifo(reqs, [1.0, 1.0, 1.0, 1.0])
    assert lat == pytest.approx([1.0, 1.9, 2.8, 1.0])
