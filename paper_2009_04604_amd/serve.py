"""Serving loop: continuous batching of simulation requests on one GPU.

A request is a lattice-Boltzmann run (geometry, tau, step count).  Requests
arrive over time; each is admitted, in arrival order, as soon as its device
footprint fits under a configured HBM budget beside the requests already
resident.  All resident requests advance together in chunks of steps through
one batched launch per step (``lbm_batch_step``: one multi-domain kernel per
lattice/storage group, replayed from a HIP graph), so requests that arrive
while others run join the running set at the next chunk boundary, and finished
ones leave it and free their memory.  The chunk is cut at the nearest
completion, so every request runs exactly its own step count.  The next chunk
is launched before the host reads back the requests the last one completed and
creates the newly admitted ones, so that host work overlaps device work; a
finished request's memory returns to the budget at the chunk boundary after its
read-back.

``Server`` holds only the scheduling; an executor object does the work:

    prepare(req)          -> job payload with .footprint (bytes); host only
    admit(payload)        -> resident handle (allocates device memory)
    step(handles, n)      -> launch n steps of every handle (asynchronous)
    sync()                -> wait for launched work
    finish(handle, req)   -> result of a finished request (reads it back)
    free(handle)

``GpuExecutor`` is the executor of the product path; tests substitute a fake
one with a fake clock.  Failures stay with their request: a request whose
preparation or admission raises is retired with an error and never holds
memory; one whose state turns non-finite is retired with an error at its
read-back; ``Server.cancel(id)`` retires a waiting or running request at the
next scheduling point (a running one after the chunk in flight).  The other
requests' results do not change.  With ``prepare_workers`` > 0 the geometry of arriving
requests is built on a thread pool (the host builder releases the GIL), so the
scheduling thread only waits for it when the request reaches the head of the
queue.  ``Server.phase`` accumulates the host seconds spent in each phase.  ``run_plain`` is the reference form: one request at a
time, in arrival order, stepped with lbm_step.
"""
import collections
import time

import numpy as np


def percentile(xs, p):
    """Nearest-rank percentile (p in [0, 100]) of a non-empty list."""
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = max(0, min(len(xs) - 1, int(np.ceil(p / 100.0 * len(xs))) - 1))
    return float(xs[k])


class Job:
    __slots__ = ("req", "payload", "handle", "footprint", "arrival", "admitted", "finished", "steps_left",
                 "result", "error", "started")

    def __init__(self, req):
        self.req = req
        self.payload = None
        self.handle = None
        self.footprint = 0
        self.arrival = float(req["arrival"])
        self.admitted = None
        self.finished = None
        self.steps_left = int(req["steps"])
        self.result = None
        self.error = None
        self.started = None                # plain form: when the server began working on it

    def record(self):
        tts = None if self.finished is None else self.finished - self.arrival
        return {"id": self.req["id"], "arrival": self.arrival, "admitted": self.admitted, "finished": self.finished,
                "time_to_solution": tts, "footprint": self.footprint, "steps": int(self.req["steps"]),
                "result": self.result, "error": self.error, "started": self.started}


class Server:
    """Continuous-batching scheduler (see the module docstring).

    hbm_budget  bytes of device memory the resident requests may hold together
    chunk       most steps launched between two scheduling points
    max_active  optional cap on the number of resident requests
    clock/sleep wall clock and wait (injectable for tests)
    trace       optional callable(event, time, info) for every scheduling event
    """

    def __init__(self, executor, hbm_budget, chunk=100, max_active=None, clock=time.perf_counter, sleep=time.sleep,
                 trace=None, prepare_workers=0):
        if hbm_budget <= 0 or chunk < 1:
            raise ValueError("hbm_budget and chunk must be positive")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.max_active = max_active
        self.clock = clock
        self.sleep = sleep
        self.trace = trace
        self.workers = int(prepare_workers)
        self.peak_bytes = 0
        self.peak_active = 0
        self.chunks = 0
        self.phase = collections.defaultdict(float)   # host seconds per scheduling phase
        self._cancel = set()

    def cancel(self, req_id):
        """Retire request req_id (waiting or running) at the next scheduling point."""
        self._cancel.add(req_id)

    def _timed(self, name, fn, *args):
        t = time.perf_counter()
        try:
            return fn(*args)
        finally:
            self.phase[name] += time.perf_counter() - t

    def _event(self, what, now, **info):
        if self.trace:
            self.trace(what, now, info)

    def run(self, requests):
        """Serve the requests (arrival times in seconds from the start of the
        call); returns one record per request, in request order."""
        jobs = [Job(r) for r in requests]
        pending = collections.deque(sorted(jobs, key=lambda j: (j.arrival, j.req["id"])))
        waiting = collections.deque()          # arrived, not admitted (FIFO)
        active = []
        pool = None
        if self.workers > 0:
            import concurrent.futures
            pool = concurrent.futures.ThreadPoolExecutor(max_workers=self.workers)
        t0 = self.clock()

        def now():
            return self.clock() - t0

        def take_arrivals():
            while pending and pending[0].arrival <= now():
                j = pending.popleft()
                # geometry is built on the host, in the pool when there is one; a
                # failure is kept with the request and raised when it is admitted
                if pool:
                    j.payload = pool.submit(self.ex.prepare, j.req)
                else:
                    try:
                        j.payload = self._timed("prepare", self.ex.prepare, j.req)
                    except Exception as e:
                        j.payload = _Failed(e)
                waiting.append(j)
                self._event("arrive", now(), id=j.req["id"])

        def ready(j):
            if isinstance(j.payload, _Failed):
                raise j.payload.exc
            if pool is not None and not isinstance(j.payload, _Done):
                j.payload = _Done(self._timed("prepare_wait", j.payload.result))
            p = j.payload.value if isinstance(j.payload, _Done) else j.payload
            j.footprint = int(p.footprint)
            return p

        try:
            self._loop(pending, waiting, active, jobs, take_arrivals, ready, now)
        finally:
            if pool is not None:
                pool.shutdown(wait=True)
        return [j.record() for j in jobs]

    def _loop(self, pending, waiting, active, jobs, take_arrivals, ready, now):
        """One iteration per chunk: wait for the chunk in flight, free what was
        read back during it, launch the next chunk, and while it runs read back
        the requests it completed and admit new ones (they join the chunk
        after)."""
        used = 0
        inflight = None           # (jobs, n) of the chunk on the device
        done = []                 # completed in the last chunk, not read back yet
        to_free = []              # read back, memory not released yet
        while pending or waiting or active or inflight or done or to_free:
            take_arrivals()
            # admission: arrival order, as long as the head fits
            while waiting:
                j = waiting[0]
                if j.req["id"] in self._cancel:
                    waiting.popleft()
                    self._retire(j, "cancelled", now())
                    continue
                try:
                    payload = ready(j)
                except Exception as e:            # preparation failed: this request only
                    waiting.popleft()
                    self._retire(j, f"preparation failed: {e}", now())
                    continue
                if j.footprint > self.budget:
                    waiting.popleft()
                    j.error = f"footprint {j.footprint} B exceeds the HBM budget {self.budget} B"
                    j.finished = now()
                    self._event("reject", now(), id=j.req["id"])
                    continue
                if used + j.footprint > self.budget:
                    break
                if self.max_active is not None and len(active) >= self.max_active:
                    break
                waiting.popleft()
                try:
                    j.handle = self._timed("admit", self.ex.admit, payload)
                except Exception as e:            # admission failed: nothing is resident
                    self._retire(j, f"admission failed: {e}", now())
                    continue
                j.payload = None
                j.admitted = now()
                used += j.footprint
                active.append(j)
                self._event("admit", now(), id=j.req["id"], used=used)
            self.peak_bytes = max(self.peak_bytes, used)
            if inflight is not None:
                self._timed("sync", self.ex.sync)
                run, n = inflight
                inflight = None
                for j in run:
                    j.steps_left -= n
                    if j.steps_left == 0:
                        done.append(j)
                # cancelled while running: out of the next chunk; memory freed at the
                # next scheduling point (no chunk in flight references it then)
                for j in active:
                    if j.steps_left > 0 and j.req["id"] in self._cancel:
                        self._retire(j, "cancelled", now())
                        to_free.append(j)
                active[:] = [j for j in active if j.steps_left > 0 and j.error is None]
            for j in to_free:
                self._timed("free", self.ex.free, j.handle)
                j.handle = None
                used -= j.footprint
                self._event("free", now(), id=j.req["id"], used=used)
            to_free = []
            if active:
                n = min(self.chunk, min(j.steps_left for j in active))
                run = list(active)
                self._timed("step_launch", self.ex.step, [j.handle for j in run], n)
                self.chunks += 1
                self.peak_active = max(self.peak_active, len(run))
                inflight = (run, n)
            # while the chunk runs: read back finished requests
            for j in done:
                j.result = self._timed("finish", self.ex.finish, j.handle, j.req)
                j.finished = now()
                if isinstance(j.result, dict) and j.result.get("unstable"):
                    j.error = "non-finite state at read-back (lbm_macros: LBM_EUNSTABLE)"
                to_free.append(j)
                self._event("finish", now(), id=j.req["id"])
            done = []
            if inflight is None and not to_free and pending and not (waiting and used + waiting[0].footprint <= self.budget):
                self.sleep(max(0.0, pending[0].arrival - now()))


    def _retire(self, j, why, t):
        j.error = why
        j.finished = t
        j.steps_left = 0
        self._event("retire", t, id=j.req["id"], why=why)


class _Failed:
    __slots__ = ("exc",)

    def __init__(self, e):
        self.exc = e


class _Done:
    __slots__ = ("value",)

    def __init__(self, v):
        self.value = v


def run_plain(executor, requests, clock=time.perf_counter, sleep=time.sleep, prepare_workers=0):
    """Reference form: one request at a time in arrival order (FIFO), each
    stepped alone to completion.  With prepare_workers > 0 the geometry of every
    request that has arrived is built on a thread pool while earlier requests
    run (the served form's preparation pool), so the plain form is not charged
    for host geometry work the served form overlaps."""
    jobs = sorted([Job(r) for r in requests], key=lambda j: (j.arrival, j.req["id"]))
    pool = None
    if prepare_workers > 0:
        import concurrent.futures
        pool = concurrent.futures.ThreadPoolExecutor(max_workers=prepare_workers)
    futures = {}
    nsub = [0]                               # jobs submitted to the pool so far, in order
    t0 = clock()

    def submit_arrived(upto):
        """Submit job upto and every later job that has already arrived."""
        if pool is None:
            return
        while nsub[0] < len(jobs) and (nsub[0] <= upto or jobs[nsub[0]].arrival <= clock() - t0):
            futures[nsub[0]] = pool.submit(executor.prepare, jobs[nsub[0]].req)
            nsub[0] += 1

    try:
        for k, j in enumerate(jobs):
            wait = j.arrival - (clock() - t0)
            if wait > 0:
                sleep(wait)
            j.started = clock() - t0
            submit_arrived(k)
            try:
                payload = futures.pop(k).result() if pool is not None else executor.prepare(j.req)
                j.footprint = int(payload.footprint)
                h = executor.admit(payload)
            except Exception as e:
                j.error = f"preparation or admission failed: {e}"
                j.finished = clock() - t0
                j.steps_left = 0
                continue
            j.admitted = clock() - t0
            submit_arrived(k)
            executor.step_alone(h, j.steps_left)
            executor.sync()
            j.result = executor.finish(h, j.req)
            if isinstance(j.result, dict) and j.result.get("unstable"):
                j.error = "non-finite state at read-back (lbm_macros: LBM_EUNSTABLE)"
            executor.free(h)
            j.steps_left = 0
            j.finished = clock() - t0
    finally:
        if pool is not None:
            pool.shutdown(wait=True)
    by_id = {j.req["id"]: j for j in jobs}
    return [by_id[r["id"]].record() for r in requests]


def busy_capacity(records):
    """Solves per second of server busy time (plain form: one request at a time,
    from when it started on a request to its read-back)."""
    busy = sum(r["finished"] - r["started"] for r in records if r["started"] is not None and r["error"] is None)
    n = sum(1 for r in records if r["started"] is not None and r["error"] is None)
    return n / busy if busy > 0 else float("inf")


def summarize(records, makespan=None):
    """solves/s over the makespan (first arrival to last completion) and
    p50 / p99 time to solution."""
    ok = [r for r in records if r["error"] is None and r["finished"] is not None]
    tts = [r["time_to_solution"] for r in ok]
    if makespan is None:
        first = min(r["arrival"] for r in records)
        last = max(r["finished"] for r in ok)
        makespan = last - first
    return {"requests": len(records), "solved": len(ok), "makespan_s": makespan,
            "solves_per_s": len(ok) / makespan if makespan > 0 else float("inf"),
            "p50_s": percentile(tts, 50), "p99_s": percentile(tts, 99), "max_s": max(tts) if tts else float("nan")}


# ---------------------------------------------------------------------------
# Executor of the product path
# ---------------------------------------------------------------------------
class _Prepared:
    __slots__ = ("req", "mask", "links", "footprint")


class GpuExecutor:
    """Requests as lbm domains on the current torch device and stream.

    storage      population storage of every request (the binding's names:
                 "f16s" / "f16s-sr" for the served form, nearest or stochastic
                 rounding of the FP16 stores; "f32" for the plain one)
    keep_fields  ids of requests whose final velocity field is returned
    autotune     run the batch autotuner once per shape class
    """

    def __init__(self, storage="f16s", keep_fields=(), autotune=False, graph=True):
        import torch
        from . import binding as B
        self.B = B
        self.storage = storage
        self.keep = set(keep_fields)
        # steps run on `stream`; domains are created and read back on `side`,
        # so that this host work overlaps the steps in flight
        self.stream = torch.cuda.Stream()
        self.side = torch.cuda.Stream()
        self.batch = B.Batch(stream=self.stream.cuda_stream)
        self.batch.set_option("graph", int(bool(graph)))
        self.batch.set_option("autotune", int(bool(autotune)))
        # device time of the step launches (HIP events on the step stream)
        self.busy_s = 0.0
        self._ev = []
        self.poison = set()                   # ids whose state is made non-finite at admission (tests)

    def footprint(self, req, mask, n_links):
        """Device bytes a request holds while resident, plus what reading its
        result back allocates: both population buffers, the segment and link
        records, the reduction partials, and at the end the residual snapshot and
        the velocity field (8 bytes per node and component each)."""
        B = self.B
        nx, ny = int(req["nx"]), int(req["ny"])
        periodic = (True, True, True) if req["kind"] == "couette" else (False, False, True)
        desc = B.make_desc("D2Q9", nx, ny, 1, req["tau"], self.storage, periodic,
                           outlet_face=None if req["kind"] == "couette" else "+x")
        pop = B.lbm_arena_bytes(desc, mask)
        rs = 8 if self.storage == "f64" else 4
        nseg = ny * ((nx + 63) // 64)
        links = n_links * (2 + 4 + 4 * rs) + nseg * 24 + 8 * 8 * (nseg // 4 + 8)
        fields = nx * ny * 2 * 8 * 2
        return int(pop + links + fields)

    def prepare(self, req):
        from . import workloads as W
        p = _Prepared()
        p.req = req
        if req["kind"] == "couette":
            p.mask, p.links = W.annulus_geometry(req)
        else:
            p.mask, p.links = W.channel_geometry(req)
        p.footprint = self.footprint(req, p.mask, len(p.links["node"]))
        return p

    def admit(self, p):
        B = self.B
        req = p.req
        side = self.side.cuda_stream
        if req["kind"] == "couette":
            d = B.Domain("D2Q9", req["nx"], req["ny"], 1, p.mask, req["tau"], storage=self.storage, stream=side)
        else:
            d = B.Domain("D2Q9", req["nx"], req["ny"], 1, p.mask, req["tau"], storage=self.storage,
                         periodic=(False, False, True), outlet_face="+x", stream=side)
        d.set_boundary_links(p.links)          # returns with the side stream drained
        if req["id"] in self.poison:
            f = d.get_state()
            f[1, np.flatnonzero(p.mask)[0]] = np.nan
            d.set_state(f)
        d.set_stream(self.stream.cuda_stream)
        d._req_mask = p.mask
        return d

    def _timed_launch(self, fn):
        import torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        fn()
        b.record(self.stream)
        self._ev.append((a, b))

    def _collect(self):
        for a, b in self._ev:
            self.busy_s += a.elapsed_time(b) / 1e3
        self._ev = []

    def step(self, handles, n):
        self._timed_launch(lambda: self.batch.step(handles, n))

    def step_alone(self, h, n):
        """Plain form: n steps of one domain, waited for."""
        self._timed_launch(lambda: h.step(n))
        self.stream.synchronize()
        self._collect()

    def sync(self):
        self.stream.synchronize()
        self._collect()

    def finish(self, h, req):
        """Read back a request whose steps have all completed (the caller has
        synchronised the step stream since its last launch), on the side stream."""
        keep = req["id"] in self.keep
        h.set_stream(self.side.cuda_stream)
        rho, u, sums, unstable = h.macros(fields=keep)
        out = {"mass": float(sums[0]), "momentum": [float(x) for x in sums[1:3]], "unstable": bool(unstable)}
        if keep:
            out["u"] = np.asarray(u, dtype=np.float64)          # (N, 2), solid nodes 0
        return out

    def free(self, h):
        h.close()

    def close(self):
        self.batch.close()
        self.stream.synchronize()
        self.side.synchronize()
