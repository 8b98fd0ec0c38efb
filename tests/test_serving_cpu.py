"""Scheduler logic of the serving loop, driven by a fake CPU executor and a
manual clock (no GPU): admission by footprint, FIFO order, continuous
batching, failure isolation, shutdown."""
import types

import pytest

from paper_2311_13182_amd.serve import Request, Scheduler


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Each request carries .fp (bytes) and .dur (seconds of virtual time);
    .fail_launch / .fail_poll force errors from the host side."""

    def __init__(self, clock):
        self.clock = clock
        self.live = {}
        self.peak_used = 0
        self.launched = []

    def footprint(self, req):
        return req.scene.fp

    def launch(self, req):
        if getattr(req.scene, "fail_launch", False):
            raise RuntimeError("launch failed (forced)")
        h = types.SimpleNamespace(req=req, t_end=self.clock() + req.scene.dur)
        self.live[id(h)] = h
        self.launched.append(req.rid)
        self.peak_used = max(self.peak_used, sum(x.req.scene.fp for x in self.live.values()))
        return h

    def poll(self, h):
        if getattr(h.req.scene, "fail_poll", False) and self.clock() >= h.t_end:
            raise RuntimeError("device error (forced)")
        return self.clock() >= h.t_end

    def collect(self, h):
        return {"cube": ("cube", h.req.rid), "n_paths": h.req.rid}

    def release(self, h):
        self.live.pop(id(h), None)


def _req(rid, fp, dur, arrival=0.0, **kw):
    return Request(rid, types.SimpleNamespace(fp=fp, dur=dur, **kw), arrival=arrival)


def _run(sch, clock, until, dt=0.001):
    while clock.t < until:
        sch.tick()
        clock.t += dt
    sch.tick()


def test_admission_respects_budget_and_fifo():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, budget_bytes=100, max_active=8, clock=clock)
    futs = [sch.submit(_req(i, fp, 0.05, arrival=0.001 * (i + 1))) for i, fp in enumerate([40, 40, 40, 10, 30])]
    _run(sch, clock, 1.0)
    res = [f.result() for f in futs]
    assert all(r.status == "ok" for r in res)
    assert ex.peak_used <= 100
    # FIFO: request 3 (small) waits behind request 2 (head of line)
    assert ex.launched == [0, 1, 2, 3, 4]
    assert res[2].t_admit >= res[0].t_done - 1e-9
    assert res[3].t_admit >= res[2].t_admit
    assert sch.used_bytes == 0


def test_continuous_batching_admits_while_others_run():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, budget_bytes=1000, max_active=4, clock=clock)
    long = sch.submit(_req(0, 100, 0.5, arrival=0.001))
    short = [sch.submit(_req(i, 100, 0.01, arrival=0.01 * i)) for i in range(1, 10)]
    _run(sch, clock, 1.0)
    L = long.result()
    S = [f.result() for f in short]
    # short requests that arrived after the long one finished before it
    assert sum(r.t_done < L.t_done for r in S) >= 8
    assert max(len([1 for r in S + [L] if r.t_admit <= t < r.t_done]) for t in [0.05, 0.1, 0.2]) <= 4


def test_max_active_slots():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_active=2, clock=clock)
    futs = [sch.submit(_req(i, 1, 0.1, arrival=0.001)) for i in range(6)]
    _run(sch, clock, 1.0)
    res = [f.result() for f in futs]
    for t in [0.05, 0.15, 0.25]:
        assert sum(r.t_admit <= t < r.t_done for r in res) <= 2


def test_oversized_request_rejected_others_served():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, budget_bytes=100, clock=clock)
    f_big = sch.submit(_req(0, 1000, 0.01, arrival=0.001))
    f_ok = sch.submit(_req(1, 50, 0.01, arrival=0.002))
    _run(sch, clock, 0.2)
    assert f_big.result().status == "rejected" and "exceeds" in f_big.result().error
    assert f_ok.result().status == "ok"


def test_failures_are_isolated_and_free_memory():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, budget_bytes=100, clock=clock)
    fa = sch.submit(_req(0, 60, 0.02, arrival=0.001, fail_launch=True))
    fb = sch.submit(_req(1, 60, 0.02, arrival=0.002, fail_poll=True))
    fc = sch.submit(_req(2, 60, 0.02, arrival=0.003))
    _run(sch, clock, 0.5)
    assert fa.result().status == "failed" and "launch failed" in fa.result().error
    assert fb.result().status == "failed" and "device error" in fb.result().error
    assert fc.result().status == "ok" and fc.result().n_paths == 2
    assert sch.used_bytes == 0 and not ex.live


def test_stop_fails_what_is_left():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, budget_bytes=100, clock=clock)
    f1 = sch.submit(_req(0, 60, 10.0, arrival=0.001))
    f2 = sch.submit(_req(1, 60, 10.0, arrival=0.002))
    _run(sch, clock, 0.01)
    sch.stop(drain=False)
    assert f1.result().status == "failed" and f2.result().status == "failed"
    assert sch.used_bytes == 0


def test_threaded_loop_with_real_clock():
    import time
    ex = FakeExecutor(time.perf_counter)
    sch = Scheduler(ex, budget_bytes=300, max_active=3)
    sch.start()
    futs = [sch.submit(_req(i, 100, 0.002)) for i in range(12)]
    res = [f.result(timeout=10) for f in futs]
    sch.stop()
    assert all(r.status == "ok" for r in res)
    assert ex.peak_used <= 300


class BatchExecutor(FakeExecutor):
    """FakeExecutor with batched launches and a cache of `resident` idle bytes
    that eviction frees."""

    def __init__(self, clock, resident=0):
        super().__init__(clock)
        self.batches = []
        self.resident = resident
        self.evicted = 0

    def launch_batch(self, reqs):
        if any(getattr(r.scene, "fail_launch", False) for r in reqs):
            raise RuntimeError("batch launch failed (forced)")
        self.batches.append([r.rid for r in reqs])
        return [FakeExecutor.launch(self, r) for r in reqs]

    def resident_bytes(self):
        return self.resident

    def evict_idle(self, nbytes):
        freed = min(nbytes, self.resident)
        self.resident -= freed
        self.evicted += freed
        return freed


def test_requests_admitted_together_share_one_batch():
    clock = Clock()
    ex = BatchExecutor(clock)
    sch = Scheduler(ex, budget_bytes=1000, max_active=8, clock=clock)
    futs = [sch.submit(_req(i, 10, 0.05, arrival=0.0005)) for i in range(5)]
    futs.append(sch.submit(_req(5, 10, 0.05, arrival=0.02)))
    _run(sch, clock, 0.5)
    assert all(f.result().status == "ok" for f in futs)
    # the five that arrived together form one batch; the late one its own
    assert ex.batches[0] == [0, 1, 2, 3, 4]
    assert [5] in ex.batches or ex.launched[-1] == 5


def test_idle_cache_bytes_reduce_the_free_budget_and_are_evicted():
    clock = Clock()
    ex = BatchExecutor(clock, resident=70)
    sch = Scheduler(ex, budget_bytes=100, max_active=8, clock=clock)
    assert sch.resident_bytes() == 70
    f = sch.submit(_req(0, 50, 0.01, arrival=0.0005))
    sch.tick()          # arrival not reached
    clock.t = 0.001
    sch.tick()          # 50 + 70 > 100: 20 bytes of idle cache are evicted to admit it
    assert ex.evicted == 20 and ex.resident == 50
    assert sch.used_bytes + sch.resident_bytes() <= 100
    _run(sch, clock, 0.1)
    assert f.result().status == "ok"


def test_cache_that_cannot_shrink_holds_admission_back():
    clock = Clock()

    class Pinned(BatchExecutor):
        def evict_idle(self, nbytes):      # nothing idle can go
            return 0

    ex = Pinned(clock, resident=70)
    sch = Scheduler(ex, budget_bytes=100, max_active=8, clock=clock)
    f = sch.submit(_req(0, 50, 0.01, arrival=0.0005))
    _run(sch, clock, 0.05)
    assert not f.done() and sch.used_bytes == 0   # 50 + 70 > 100: waits
    ex.resident = 10
    _run(sch, clock, 0.1)
    assert f.result().status == "ok"


def test_failed_batch_falls_back_to_single_launches():
    clock = Clock()
    ex = BatchExecutor(clock)
    sch = Scheduler(ex, budget_bytes=1000, max_active=8, clock=clock)
    fa = sch.submit(_req(0, 10, 0.01, arrival=0.0005, fail_launch=True))
    fb = sch.submit(_req(1, 10, 0.01, arrival=0.0005))
    _run(sch, clock, 0.2)
    assert fa.result().status == "failed" and "launch failed" in fa.result().error
    assert fb.result().status == "ok"
    assert sch.used_bytes == 0


def test_request_that_cannot_be_sized_fails_alone():
    clock = Clock()

    class Picky(FakeExecutor):
        def footprint(self, req):
            if getattr(req.scene, "unsizable", False):
                raise ValueError("no footprint (forced)")
            return req.scene.fp

    ex = Picky(clock)
    sch = Scheduler(ex, budget_bytes=100, clock=clock)
    fa = sch.submit(_req(0, 10, 0.01, arrival=0.0005, unsizable=True))
    fb = sch.submit(_req(1, 10, 0.01, arrival=0.0006))
    _run(sch, clock, 0.1)
    assert fa.result().status == "failed" and "no footprint" in fa.result().error
    assert fb.result().status == "ok"
    assert sch.used_bytes == 0 and sch.idle()


def test_idle_is_false_while_a_batch_is_being_launched():
    """A request taken off the queue counts as work until it is active, so a
    draining stop() cannot end the loop between the two."""
    clock = Clock()
    seen = []

    class Watch(BatchExecutor):
        def launch_batch(self, reqs):
            seen.append(sch.idle())
            return super().launch_batch(reqs)

    ex = Watch(clock)
    sch = Scheduler(ex, budget_bytes=1000, clock=clock)
    futs = [sch.submit(_req(i, 10, 0.01, arrival=0.0005)) for i in range(3)]
    _run(sch, clock, 0.1)
    assert seen == [False]
    assert all(f.result().status == "ok" for f in futs)


def test_request_that_never_completes_times_out_and_frees_memory():
    clock = Clock()

    class Stuck(FakeExecutor):
        def poll(self, h):
            return False if getattr(h.req.scene, "stuck", False) else super().poll(h)

    ex = Stuck(clock)
    sch = Scheduler(ex, budget_bytes=100, clock=clock, request_timeout=0.05)
    fa = sch.submit(_req(0, 60, 0.01, arrival=0.0005, stuck=True))
    fb = sch.submit(_req(1, 60, 0.01, arrival=0.0006))   # waits for the stuck one's memory
    _run(sch, clock, 0.2)
    ra, rb = fa.result(), fb.result()
    assert ra.status == "failed" and "TimeoutError" in ra.error
    assert rb.status == "ok" and rb.t_admit >= ra.t_done - 1e-9
    assert sch.used_bytes == 0 and not ex.live


def test_admissions_of_one_tick_are_launched_in_groups_of_max_batch():
    clock = Clock()
    ex = BatchExecutor(clock)
    sch = Scheduler(ex, budget_bytes=10 ** 6, max_active=64, clock=clock, max_batch=4)
    futs = [sch.submit(_req(i, 10, 0.01, arrival=0.0005)) for i in range(10)]
    _run(sch, clock, 0.2)
    assert all(f.result().status == "ok" for f in futs)
    assert ex.batches == [[0, 1, 2, 3], [4, 5, 6, 7], [8, 9]]


class SlowCollectExecutor(BatchExecutor):
    """BatchExecutor whose collect takes wall time, may fail (.fail_collect),
    and records the thread it ran on and whether a handle was released while
    its collect was still running."""

    def __init__(self, clock, collect_s=0.003):
        super().__init__(clock)
        import threading
        self.collect_s = collect_s
        self.threads = set()
        self.in_collect = set()
        self.released_early = []
        self.lock = threading.Lock()

    def collect(self, h):
        import threading
        import time
        with self.lock:
            self.threads.add(threading.current_thread().name)
            self.in_collect.add(id(h))
        try:
            time.sleep(self.collect_s)
            if getattr(h.req.scene, "fail_collect", False):
                raise RuntimeError("copy failed (forced)")
            return FakeExecutor.collect(self, h)
        finally:
            with self.lock:
                self.in_collect.discard(id(h))

    def release(self, h):
        with self.lock:
            if id(h) in self.in_collect:
                self.released_early.append(h.req.rid)
        FakeExecutor.release(self, h)


def test_collect_workers_copy_results_off_the_scheduler_thread():
    import time
    ex = SlowCollectExecutor(time.perf_counter)
    sch = Scheduler(ex, budget_bytes=10 ** 6, max_active=16, max_batch=4, collect_workers=2)
    sch.start()
    futs = [sch.submit(_req(i, 100, 0.001, fail_collect=(i == 5))) for i in range(24)]
    res = [f.result(timeout=10) for f in futs]
    sch.stop()
    assert [r.rid for r in res] == list(range(24))
    assert [r.status for r in res] == ["failed" if i == 5 else "ok" for i in range(24)]
    assert "copy failed" in res[5].error
    assert all(r.cube == ("cube", r.rid) and r.n_paths == r.rid for r in res if r.status == "ok")
    assert ex.threads and all(t.startswith("sbr-collect") for t in ex.threads)
    assert ex.released_early == [] and not ex.live and sch.used_bytes == 0


def test_stop_waits_for_copies_in_flight():
    import time
    ex = SlowCollectExecutor(time.perf_counter, collect_s=0.2)
    sch = Scheduler(ex, budget_bytes=10 ** 6, max_active=4, collect_workers=1)
    futs = [sch.submit(_req(i, 100, 0.0)) for i in range(2)]
    sch.tick()                 # admit and launch both
    time.sleep(0.001)
    sch.tick()                 # both done on the device: their copies start
    assert len(sch._active) == 2 and all(item[5] is not None for item in sch._active)
    sch.stop(drain=False)
    res = [f.result(timeout=10) for f in futs]
    assert [r.status for r in res] == ["failed", "failed"]
    assert all("scheduler stopped" in r.error for r in res)
    assert ex.released_early == [] and not ex.live and sch.used_bytes == 0
