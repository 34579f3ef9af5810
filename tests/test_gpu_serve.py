"""Serving loop on the GPU: requests served in a continuously batched mix end
in the same state as when each runs alone (bit for bit: the batched kernel does
the same per-node arithmetic), memory stays under the budget, and requests are
admitted while others run.  A virtual clock that advances with every launched
step makes the interleaving independent of the GPU's speed."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


class StepClock:
    """Virtual time: dt seconds per launched step."""

    def __init__(self, dt=1e-3):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        return self.t

    def sleep(self, s):
        self.t += max(0.0, s)


class Clocked:
    """Executor wrapper that advances the virtual clock on every launch."""

    def __init__(self, ex, clock):
        self.ex, self.clock = ex, clock

    def __getattr__(self, k):
        return getattr(self.ex, k)

    def step(self, handles, n):
        self.ex.step(handles, n)
        self.clock.t += n * self.clock.dt


def _requests():
    reqs = synth.request_stream(n_requests=7, l_min=64, l_max=144, seed=13, steps=240)
    for k, r in enumerate(reqs):
        r["arrival"] = 0.05 * k              # a new request every 50 virtual steps
        r["steps"] = 240 - 20 * (k % 3)
    return reqs


@pytest.mark.parametrize("storage", ["f16s", "f32"])
def test_served_mix_equals_alone(gpu_lib, storage):
    from paper_2009_04604_amd import serve
    print("case served mix", storage, flush=True)
    reqs = _requests()
    ids = [r["id"] for r in reqs]
    clk = StepClock()
    ex = serve.GpuExecutor(storage=storage, keep_fields=ids)
    events = []
    srv = serve.Server(Clocked(ex, clk), hbm_budget=5 * 2**20, chunk=40, clock=clk, sleep=clk.sleep,
                       trace=lambda e, t, info: events.append((e, t, info)))
    recs = srv.run(reqs)
    ex.close()
    assert all(r["error"] is None for r in recs)
    assert srv.peak_bytes <= 5 * 2**20
    assert srv.peak_active >= 2
    # some request was admitted while an earlier one was still running
    assert any(b["admitted"] > a["admitted"] and b["admitted"] < a["finished"] for a in recs for b in recs)
    alone = serve.GpuExecutor(storage=storage, keep_fields=ids)
    for r, q in zip(recs, reqs):
        h = alone.admit(alone.prepare(q))
        alone.step_alone(h, q["steps"])
        res = alone.finish(h, q)
        alone.free(h)
        assert np.array_equal(res["u"], r["result"]["u"]), f"request {q['id']}"
        assert res["mass"] == r["result"]["mass"]
        assert not r["result"]["unstable"]
    alone.close()


def test_served_error_against_fp64_is_stated(gpu_lib):
    """FP16-shifted served results against the same request in FP64 (the FP64
    path matches the FP64 oracle to 1e-12): relative L2 velocity error."""
    from paper_2009_04604_amd import serve
    reqs = _requests()[:2]
    errs = []
    for q in reqs:
        out = {}
        for st in ("f16s", "f64"):
            ex = serve.GpuExecutor(storage=st, keep_fields=[q["id"]])
            h = ex.admit(ex.prepare(q))
            ex.step_alone(h, q["steps"])
            out[st] = ex.finish(h, q)["u"]
            ex.free(h)
            ex.close()
        e = np.linalg.norm(out["f16s"] - out["f64"]) / np.linalg.norm(out["f64"])
        print("request", q["id"], q["kind"], q["L"], "E(f16s vs f64)", e, flush=True)
        errs.append(e)
    assert max(errs) < 0.03


def test_failing_and_cancelled_requests_retire_alone(gpu_lib):
    """In a served mix: a request whose state is made non-finite at admission is
    retired with an error at its read-back (lbm_macros reports LBM_EUNSTABLE), a
    request the library refuses (tau <= 1/2) is retired at admission, and one
    is cancelled while running; every other request ends bit-identical to the
    same request run alone, and the budget is released."""
    from paper_2009_04604_amd import serve
    print("case served mix with failures", flush=True)
    reqs = _requests()
    reqs[2]["tau"] = 0.45                    # refused by lbm_init_domain
    ids = [r["id"] for r in reqs]
    clk = StepClock()
    ex = serve.GpuExecutor(storage="f32", keep_fields=ids)
    ex.poison = {reqs[4]["id"]}
    victim = reqs[1]["id"]
    seen = {"admitted": False, "chunks": 0}

    class CancelAfterTwoChunks(Clocked):
        """Cancels the victim once two chunks have run since its admission (it
        needs at least five), so it is cancelled while running."""

        def step(self, handles, n):
            super().step(handles, n)
            if seen["admitted"]:
                seen["chunks"] += 1
                if seen["chunks"] == 2:
                    srv.cancel(victim)

    srv = serve.Server(CancelAfterTwoChunks(ex, clk), hbm_budget=5 * 2**20, chunk=40, clock=clk, sleep=clk.sleep)

    def trace(what, t, info):
        if what == "admit" and info["id"] == victim:
            seen["admitted"] = True
    srv.trace = trace
    recs = srv.run(reqs)
    ex.close()
    assert "admission failed" in recs[2]["error"]
    assert "non-finite" in recs[4]["error"] and recs[4]["result"]["unstable"]
    assert seen["chunks"] >= 2 and recs[1]["error"] == "cancelled"
    alone = serve.GpuExecutor(storage="f32", keep_fields=ids)
    for k in (0, 3, 5, 6):
        q, r = reqs[k], recs[k]
        assert r["error"] is None
        h = alone.admit(alone.prepare(q))
        alone.step_alone(h, q["steps"])
        res = alone.finish(h, q)
        alone.free(h)
        assert np.array_equal(res["u"], r["result"]["u"]), f"request {q['id']}"
    alone.close()
