"""Scheduling logic of the serving loop (paper_2009_04604_amd.serve) on the CPU:
a fake executor with a cost model and a fake clock stand in for the GPU."""
import numpy as np
import pytest

from paper_2009_04604_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeExecutor:
    """Cost of a launch of n steps over a set of domains: n * (overhead + sum of
    per-domain work); bytes per node fixed."""

    def __init__(self, clock, bytes_per_node=10, overhead=1e-3, work_per_node=1e-8):
        self.clock = clock
        self.bpn = bytes_per_node
        self.overhead = overhead
        self.wpn = work_per_node
        self.resident = 0
        self.peak = 0
        self.log = []
        self.steps = {}
        self.admit_order = []

    class P:
        def __init__(self, req, fp):
            self.req, self.footprint = req, fp

    def prepare(self, req):
        return self.P(req, req["nx"] * req["ny"] * self.bpn)

    def admit(self, p):
        self.resident += p.footprint
        self.peak = max(self.peak, self.resident)
        self.admit_order.append(p.req["id"])
        h = {"id": p.req["id"], "nodes": p.req["nx"] * p.req["ny"], "fp": p.footprint}
        self.steps[h["id"]] = []
        return h

    def step(self, handles, n):
        self.log.append((self.clock(), [h["id"] for h in handles], n))
        for h in handles:
            self.steps[h["id"]].append(n)
        self.clock.t += n * (self.overhead + self.wpn * sum(h["nodes"] for h in handles))

    def step_alone(self, h, n):
        self.step([h], n)

    def sync(self):
        pass

    def finish(self, h, req):
        return {"steps_done": sum(self.steps[h["id"]])}

    def free(self, h):
        self.resident -= h["fp"]


def _reqs(n=24, seed=3, rate=50.0, steps=(200, 600)):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        L = int(rng.integers(64, 257))
        out.append({"id": k, "nx": L, "ny": L, "arrival": t, "steps": int(rng.integers(*steps))})
    return out


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == 50
    assert serve.percentile(xs, 99) == 99
    assert serve.percentile(xs, 100) == 100
    assert serve.percentile([5.0], 99) == 5.0
    assert serve.percentile([3, 1, 2], 50) == 2


def test_every_request_runs_exactly_its_steps_in_chunks():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _reqs()
    srv = serve.Server(ex, hbm_budget=4_000_000, chunk=64, clock=clk, sleep=clk.sleep)
    recs = srv.run(reqs)
    for r, q in zip(recs, reqs):
        assert r["error"] is None
        assert r["result"]["steps_done"] == q["steps"]
        assert all(0 < n <= 64 for n in ex.steps[q["id"]])
        assert r["admitted"] >= q["arrival"] - 1e-12 and r["finished"] > r["admitted"]


def test_budget_is_never_exceeded_and_admission_is_fifo():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _reqs(n=40, rate=500.0)
    budget = 1_500_000
    srv = serve.Server(ex, hbm_budget=budget, chunk=50, clock=clk, sleep=clk.sleep)
    recs = srv.run(reqs)
    assert ex.peak <= budget
    assert srv.peak_bytes <= budget
    assert ex.admit_order == sorted(ex.admit_order, key=lambda i: (reqs[i]["arrival"], i))
    assert ex.resident == 0
    assert all(r["error"] is None for r in recs)


def test_continuous_batching_admits_while_others_run():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = [{"id": 0, "nx": 100, "ny": 100, "arrival": 0.0, "steps": 1000},
            {"id": 1, "nx": 100, "ny": 100, "arrival": 0.05, "steps": 100}]
    srv = serve.Server(ex, hbm_budget=10**9, chunk=50, clock=clk, sleep=clk.sleep)
    recs = srv.run(reqs)
    # request 1 joined the running set and finished long before request 0
    assert recs[1]["admitted"] < recs[0]["finished"]
    assert recs[1]["finished"] < recs[0]["finished"]
    assert any(ids == [0, 1] for _, ids, _ in ex.log)
    assert srv.peak_active == 2


def test_oversized_request_is_rejected_and_head_of_line_waits():
    clk = FakeClock()
    ex = FakeExecutor(clk, bytes_per_node=100)
    reqs = [{"id": 0, "nx": 100, "ny": 100, "arrival": 0.0, "steps": 300},      # 1 MB
            {"id": 1, "nx": 200, "ny": 200, "arrival": 0.001, "steps": 100},    # 4 MB: too big
            {"id": 2, "nx": 90, "ny": 90, "arrival": 0.002, "steps": 100},      # 0.81 MB: must wait for 0
            {"id": 3, "nx": 10, "ny": 10, "arrival": 0.003, "steps": 100}]      # tiny, but behind 2 (FIFO)
    srv = serve.Server(ex, hbm_budget=1_500_000, chunk=100, clock=clk, sleep=clk.sleep)
    recs = srv.run(reqs)
    assert recs[1]["error"] is not None and recs[1]["result"] is None
    assert recs[2]["admitted"] >= recs[0]["finished"]
    assert recs[3]["admitted"] >= recs[2]["admitted"]
    assert ex.peak <= 1_500_000


def test_max_active_cap():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    srv = serve.Server(ex, hbm_budget=10**9, chunk=30, max_active=3, clock=clk, sleep=clk.sleep)
    srv.run(_reqs(n=12, rate=1e4))
    assert srv.peak_active == 3
    assert max(len(ids) for _, ids, _ in ex.log) == 3


def test_batched_beats_plain_when_launch_overhead_matters():
    reqs = _reqs(n=30, rate=20.0, steps=(300, 400))
    clk = FakeClock()
    served = serve.Server(FakeExecutor(clk), hbm_budget=10**9, chunk=100, clock=clk, sleep=clk.sleep).run(reqs)
    clk2 = FakeClock()
    plain = serve.run_plain(FakeExecutor(clk2), reqs, clock=clk2, sleep=clk2.sleep)
    s, p = serve.summarize(served), serve.summarize(plain)
    assert s["solved"] == p["solved"] == 30
    assert s["p99_s"] < p["p99_s"]
    assert s["solves_per_s"] > p["solves_per_s"]


def test_idle_server_waits_for_arrivals():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = [{"id": 0, "nx": 64, "ny": 64, "arrival": 5.0, "steps": 10}]
    recs = serve.Server(ex, hbm_budget=10**9, clock=clk, sleep=clk.sleep).run(reqs)
    assert recs[0]["admitted"] >= 5.0
    assert recs[0]["time_to_solution"] == pytest.approx(10 * (1e-3 + 1e-8 * 64 * 64))


def test_prepare_pool_gives_the_same_schedule():
    reqs = _reqs(n=20, rate=200.0)
    out = []
    for workers in (0, 3):
        clk = FakeClock()
        ex = FakeExecutor(clk)
        srv = serve.Server(ex, hbm_budget=2_000_000, chunk=40, clock=clk, sleep=clk.sleep, prepare_workers=workers)
        recs = srv.run(reqs)
        out.append(([(r["admitted"], r["finished"]) for r in recs], ex.admit_order))
        assert set(srv.phase) >= {"admit", "step_launch", "sync", "finish", "free"}
    assert out[0] == out[1]


def test_plain_busy_capacity():
    reqs = _reqs(n=10, rate=5.0)
    clk = FakeClock()
    recs = serve.run_plain(FakeExecutor(clk), reqs, clock=clk, sleep=clk.sleep)
    service = [q["steps"] * (1e-3 + 1e-8 * q["nx"] * q["ny"]) for q in reqs]
    assert serve.busy_capacity(recs) == pytest.approx(len(reqs) / sum(service))


class FailingExecutor(FakeExecutor):
    """Preparation of bad_prepare, admission of bad_admit raise; nan_ids read back
    as non-finite."""

    def __init__(self, clock, bad_prepare=(), bad_admit=(), nan_ids=()):
        super().__init__(clock)
        self.bad_prepare, self.bad_admit, self.nan_ids = set(bad_prepare), set(bad_admit), set(nan_ids)

    def prepare(self, req):
        if req["id"] in self.bad_prepare:
            raise ValueError("tau must be finite and > 0.5")
        return super().prepare(req)

    def admit(self, p):
        if p.req["id"] in self.bad_admit:
            raise RuntimeError("liblbm error -2: hipMalloc: out of memory")
        return super().admit(p)

    def finish(self, h, req):
        out = super().finish(h, req)
        out["unstable"] = req["id"] in self.nan_ids
        return out


def test_failing_requests_are_retired_alone():
    """A request that cannot be prepared, one that cannot be admitted and one
    whose state turns non-finite are retired with an error; every other request
    runs exactly as in a run without them, and no memory stays held."""
    reqs = _reqs(n=16, rate=300.0)
    clk = FakeClock()
    ok = serve.Server(FakeExecutor(clk), hbm_budget=10**9, chunk=50, clock=clk, sleep=clk.sleep).run(reqs)
    clk2 = FakeClock()
    ex = FailingExecutor(clk2, bad_prepare=[3], bad_admit=[7], nan_ids=[11])
    recs = serve.Server(ex, hbm_budget=10**9, chunk=50, clock=clk2, sleep=clk2.sleep).run(reqs)
    assert "preparation failed" in recs[3]["error"] and recs[3]["admitted"] is None
    assert "admission failed" in recs[7]["error"] and recs[7]["admitted"] is None
    assert "non-finite" in recs[11]["error"]
    for k in set(range(16)) - {3, 7, 11}:
        assert recs[k]["error"] is None
        assert recs[k]["result"]["steps_done"] == reqs[k]["steps"] == ok[k]["result"]["steps_done"]
    assert ex.resident == 0


def test_cancel_running_and_waiting_requests():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = [{"id": 0, "nx": 100, "ny": 100, "arrival": 0.0, "steps": 2000},
            {"id": 1, "nx": 100, "ny": 100, "arrival": 0.0, "steps": 300},
            {"id": 2, "nx": 100, "ny": 100, "arrival": 0.0, "steps": 300}]
    srv = serve.Server(ex, hbm_budget=250_000, chunk=50, clock=clk, sleep=clk.sleep)   # room for two

    def trace(what, t, info):
        if what == "admit" and info["id"] == 1:
            srv.cancel(0)                         # running: leaves after the chunk in flight
            srv.cancel(2)                         # waiting: never admitted
    srv.trace = trace
    recs = srv.run(reqs)
    assert recs[0]["error"] == "cancelled" and sum(ex.steps[0]) < 2000
    assert recs[2]["error"] == "cancelled" and recs[2]["admitted"] is None
    assert recs[1]["error"] is None and recs[1]["result"]["steps_done"] == 300
    assert ex.resident == 0


def test_plain_prefetch_pool_same_results():
    reqs = _reqs(n=12, rate=50.0)
    out = []
    for workers in (0, 3):
        clk = FakeClock()
        recs = serve.run_plain(FakeExecutor(clk), reqs, clock=clk, sleep=clk.sleep, prepare_workers=workers)
        out.append([(r["id"], r["result"]["steps_done"], r["finished"]) for r in recs])
    assert out[0] == out[1]
    clk = FakeClock()
    recs = serve.run_plain(FailingExecutor(clk, bad_prepare=[4]), reqs, clock=clk, sleep=clk.sleep, prepare_workers=2)
    assert "failed" in recs[4]["error"] and all(r["error"] is None for k, r in enumerate(recs) if k != 4)
