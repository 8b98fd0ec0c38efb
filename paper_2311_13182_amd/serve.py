"""Serving loop: a persistent scheduler that runs forward and forward+backward
simulations of many requests on one GPU with continuous batching.

* Admission by device-memory footprint: a request is admitted when its
  estimated footprint fits the free part of the budget (FIFO order, a request
  larger than the whole budget is rejected).
* Continuous batching: an admitted request's whole pipeline (mesh upload, BVH
  build, trace, synthesis, and for forward+backward the loss entry and the
  adjoint) is enqueued at once on one of several HIP streams; requests that
  arrive while others run are admitted as soon as memory and slots free up,
  so their kernels overlap other requests' kernels on the device.
* BVHs and meshes stay resident for the life of a request, and repeated
  meshes reuse a cached device copy (LRU keyed by the mesh bytes).
* Each request's launch shapes depend only on its own sizes, so its forward
  result is bit-identical alone and in the mix (the backward differs only in
  the order of floating-point atomics).

The scheduler is independent of the device: `Scheduler` drives any object
with the executor interface (`footprint`, `launch`, `poll`, `collect`,
`release`), which the tests replace with a CPU fake.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import hashlib
import json
import threading
import time
from typing import Any, Deque, Dict, List, Optional

import numpy as np

from . import scenes as S


@dataclasses.dataclass
class Request:
    rid: int
    scene: S.Scene
    backward: bool = False
    target: Optional[np.ndarray] = None      # complex64 [V,C,S] for backward requests
    arrival: float = 0.0                     # seconds, scheduler clock (0 = now)


@dataclasses.dataclass
class Result:
    rid: int
    status: str                              # "ok" | "failed" | "rejected"
    cube: Optional[np.ndarray] = None
    grad: Optional[np.ndarray] = None
    n_paths: int = -1
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    footprint: int = 0
    error: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Scheduler:
    """Admission + continuous batching over an executor.  Thread-safe submit."""

    def __init__(self, executor, budget_bytes: int, max_active: int = 16, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.clock = clock
        self.t0 = clock()
        self._pending: Deque = collections.deque()
        self._active: List = []
        self._used = 0
        self._footprints: Dict[int, int] = {}
        self._lock = threading.Lock()
        self._stop = threading.Event()
        self._thread: Optional[threading.Thread] = None
        self.log: List[Result] = []

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> concurrent.futures.Future:
        fut: concurrent.futures.Future = concurrent.futures.Future()
        with self._lock:
            if req.arrival <= 0.0:
                req.arrival = self.now()
            self._pending.append((req, fut))
        return fut

    # one scheduling round: completions first, then admissions
    def tick(self) -> bool:
        progressed = False
        still = []
        for item in self._active:
            req, fut, h, fp, t_admit = item
            try:
                done = self.ex.poll(h)
            except Exception as e:   # device-side failure of this request only
                self._finish(req, fut, h, fp, t_admit, None, e)
                progressed = True
                continue
            if done:
                try:
                    out = self.ex.collect(h)
                    self._finish(req, fut, h, fp, t_admit, out, None)
                except Exception as e:
                    self._finish(req, fut, h, fp, t_admit, None, e)
                progressed = True
            else:
                still.append(item)
        self._active = still
        now = self.now()
        while True:
            with self._lock:
                if not self._pending or self._pending[0][0].arrival > now:
                    break
                req, fut = self._pending[0]
                fp = self._footprints.get(req.rid)
                if fp is None:
                    fp = self._footprints[req.rid] = self.ex.footprint(req)
                if fp > self.budget:
                    self._pending.popleft()
                    res = Result(req.rid, "rejected", t_arrival=req.arrival, t_done=now, footprint=fp,
                                 error=f"footprint {fp} B exceeds the budget {self.budget} B")
                    self.log.append(res)
                    fut.set_result(res)
                    progressed = True
                    continue
                if self._used + fp > self.budget or len(self._active) >= self.max_active:
                    break
                self._pending.popleft()
            t_admit = self.now()
            try:
                h = self.ex.launch(req)
            except Exception as e:
                res = Result(req.rid, "failed", t_arrival=req.arrival, t_admit=t_admit, t_done=self.now(),
                             footprint=fp, error=repr(e))
                self.log.append(res)
                fut.set_result(res)
                progressed = True
                continue
            self._used += fp
            self._active.append((req, fut, h, fp, t_admit))
            progressed = True
        return progressed

    def _finish(self, req, fut, h, fp, t_admit, out, err):
        try:
            self.ex.release(h)
        finally:
            self._used -= fp
        if err is None:
            res = Result(req.rid, "ok", cube=out.get("cube"), grad=out.get("grad"), n_paths=out.get("n_paths", -1),
                         t_arrival=req.arrival, t_admit=t_admit, t_done=self.now(), footprint=fp)
        else:
            res = Result(req.rid, "failed", t_arrival=req.arrival, t_admit=t_admit, t_done=self.now(),
                         footprint=fp, error=repr(err))
        self.log.append(res)
        fut.set_result(res)

    def idle(self) -> bool:
        with self._lock:
            return not self._pending and not self._active

    @property
    def used_bytes(self) -> int:
        return self._used

    def start(self):
        self._stop.clear()
        self._thread = threading.Thread(target=self._loop, name="sbr-scheduler", daemon=True)
        self._thread.start()

    def _loop(self):
        while not self._stop.is_set():
            if not self.tick():
                time.sleep(0.0002)

    def stop(self, drain: bool = True, timeout: float = 600.0):
        if drain:
            t_end = time.perf_counter() + timeout
            while not self.idle() and time.perf_counter() < t_end:
                time.sleep(0.001)
        self._stop.set()
        if self._thread:
            self._thread.join()
        # anything left is failed explicitly (never silently dropped)
        for req, fut, h, fp, t_admit in self._active:
            self._finish(req, fut, h, fp, t_admit, None, RuntimeError("scheduler stopped"))
        self._active = []
        with self._lock:
            while self._pending:
                req, fut = self._pending.popleft()
                res = Result(req.rid, "failed", t_arrival=req.arrival, t_done=self.now(), error="scheduler stopped")
                self.log.append(res)
                fut.set_result(res)


# --------------------------------------------------------------------------- GPU executor
def request_footprint(scene: S.Scene, backward: bool) -> int:
    """Device bytes a request holds while active: mesh, BVH, hit records,
    scratch, IF cube (x3 for forward+backward: cube, target, gradient) and
    vertex gradients."""
    from . import sbr as B
    from . import _lib as L
    g, rd, ch = scene.grid, scene.radar, scene.chirp
    V, C, Sn, R, K = rd.n_virtual, ch.n_chirps, ch.n_samples, g.n_rays, g.max_bounces
    mesh = scene.nv * 12 + scene.nf * 12
    bvh = B.sbr_bvh_bytes(scene.nf)
    ops = [L.SBR_OP_SYNTH] + ([L.SBR_OP_BACKWARD] if backward else [])
    scratch = max(B.sbr_scratch_bytes(op, None, g, rd, ch) for op in ops)
    scratch = max(scratch, 64 * scene.nf + (1 << 20), 16 * 64 * C * Sn + 1024)   # BVH build, radar cube
    hits = R * K * 17
    cube = V * C * Sn * 8 * (3 if backward else 1)
    grads = scene.nv * 12 if backward else 0
    return int(mesh + bvh + scratch + hits + cube + grads + (1 << 20))


def _mesh_key(scene: S.Scene) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(scene.verts).tobytes())
    h.update(np.ascontiguousarray(scene.faces).tobytes())
    return h.hexdigest()


class GPUExecutor:
    """Runs each request's pipeline on one of `n_streams` HIP streams."""

    def __init__(self, device="cuda", n_streams: int = 4, cache_meshes: int = 8):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]  # default priority
        self.next = 0
        self.cache: "collections.OrderedDict[str, Any]" = collections.OrderedDict()
        self.cache_meshes = cache_meshes

    def footprint(self, req: Request) -> int:
        return request_footprint(req.scene, req.backward)

    def launch(self, req: Request):
        torch = self.torch
        from .sbr import DeviceMesh, Simulator
        st = self.streams[self.next % len(self.streams)]
        self.next += 1
        out: Dict[str, Any] = {"stream": st}
        with torch.cuda.stream(st):
            key = _mesh_key(req.scene)
            cached = self.cache.get(key)
            if cached is not None:       # resident mesh + BVH of an identical mesh
                self.cache.move_to_end(key)
                mesh, bvh = cached
                for t in (mesh.verts, mesh.faces, bvh):
                    t.record_stream(st)
                sim = Simulator(req.scene, self.device, mesh=mesh, bvh=bvh)
            else:
                mesh = DeviceMesh.from_scene(req.scene, self.device, non_blocking=True)
                sim = Simulator(req.scene, self.device, mesh=mesh)
                sim.build()
                self.cache[key] = (sim.mesh, sim.bvh)
                while len(self.cache) > self.cache_meshes:
                    self.cache.popitem(last=False)
            sim.trace()
            cube = sim.synth()
            out["sim"], out["cube"] = sim, cube
            # the synthesis leaves the path count in the scratch buffer
            out["n_paths_dev"] = sim.scratch[:4].view(torch.int32).clone()
            if req.backward:
                th = torch.from_numpy(np.ascontiguousarray(req.target, dtype=np.complex64)).pin_memory()
                tgt = th.to(self.device, non_blocking=True)
                out["target_staging"] = th
                grad, _ = sim.loss_grad(cube, tgt)
                out["grad"] = sim.backward(grad)
                out["grad_host"] = torch.empty(out["grad"].shape, dtype=torch.float32, pin_memory=True)
                out["grad_host"].copy_(out["grad"], non_blocking=True)
            out["cube_host"] = torch.empty(cube.shape, dtype=torch.float32, pin_memory=True)
            out["cube_host"].copy_(cube, non_blocking=True)
            out["np_host"] = torch.empty(1, dtype=torch.int32, pin_memory=True)
            out["np_host"].copy_(out["n_paths_dev"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
            out["event"] = ev
        return out

    def poll(self, h) -> bool:
        return h["event"].query()

    def collect(self, h) -> Dict[str, Any]:
        h["event"].synchronize()
        res = {"cube": h["cube_host"].numpy().view(np.complex64).reshape(h["cube"].shape[:-1]).copy(),
               "n_paths": int(h["np_host"][0])}
        if "grad_host" in h:
            res["grad"] = h["grad_host"].numpy().copy()
        return res

    def release(self, h):
        h.clear()


def run_sequential(executor, requests: List[Request]) -> List[Result]:
    """One request at a time, in arrival order, waiting for each to finish."""
    out = []
    t0 = time.perf_counter()
    for req in requests:
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        ta = time.perf_counter() - t0
        h = executor.launch(req)
        while not executor.poll(h):
            time.sleep(0.0001)
        r = executor.collect(h)
        executor.release(h)
        out.append(Result(req.rid, "ok", cube=r["cube"], grad=r.get("grad"), n_paths=r["n_paths"],
                          t_arrival=req.arrival, t_admit=ta, t_done=time.perf_counter() - t0))
    return out


def summarize(results: List[Result], wall: float) -> Dict[str, float]:
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    return {"requests": len(results), "ok": len(ok), "wall_s": wall, "throughput_rps": len(ok) / wall,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3), "p99_latency_ms": float(np.percentile(lat, 99) * 1e3)}


def serving_benchmark(n: int = 512, seed: int = 5, budget_gb: float = 64.0, n_streams: int = 4,
                      max_active: int = 16, grids=(256, 512, 1024, 2048), nf_range=(1000, 200000),
                      phases=(("main", 1.25), ("low", 0.5)), quiet: bool = False):
    """Sequential FIFO solves vs the continuous-batching server on the same
    Poisson request stream (QPS = 1.25 x the measured sequential rate)."""
    import sys
    import torch

    def say(msg):
        if not quiet:
            print(f"[serving] {msg}", file=sys.stderr, flush=True)

    reqs = S.serving_requests(n=n, qps=1.0, seed=seed, grids=grids, nf_range=nf_range)
    say(f"{n} requests generated")
    ex = GPUExecutor(n_streams=n_streams)
    # targets of the backward requests: jittered-mesh cubes (untimed)
    for r in reqs:
        if r.backward:
            h = ex.launch(Request(-1, S.jitter(r.scene, 2e-3, 33 + r.rid)))
            r.target = ex.collect(h)["cube"]
            ex.release(h)
    plain = [Request(r.rid, r.scene, r.backward, r.target, 0.0) for r in reqs]
    # warm-up (library load, allocator)
    h = ex.launch(plain[0])
    ex.collect(h)
    ex.release(h)
    torch.cuda.synchronize()
    say("targets ready")
    t0 = time.perf_counter()
    seq_all = run_sequential(ex, plain)
    seq_wall = time.perf_counter() - t0
    mu = n / seq_wall
    say(f"sequential service rate {mu:.2f} req/s")
    out = {"mu_seq_rps": mu, "n_backward": sum(r.backward for r in reqs)}
    for tag, factor in phases:
        qps = factor * mu
        rng = np.random.default_rng(seed + 1)
        arr = np.cumsum(rng.exponential(1.0 / qps, size=n))
        timed = [Request(r.rid, r.scene, r.backward, r.target, float(a)) for r, a in zip(reqs, arr)]
        seq = run_sequential(ex, timed)
        seq_w = max(r.t_done for r in seq)
        sch = Scheduler(ex, int(budget_gb * (1 << 30)), max_active=max_active)
        futs = [sch.submit(r) for r in timed]
        sch.t0 = time.perf_counter()
        sch.start()
        res = [f.result() for f in futs]
        sch.stop()
        srv_w = max(r.t_done for r in res)
        out[tag] = {"qps": qps, "sequential": summarize(seq, seq_w), "server": summarize(res, srv_w)}
        say(f"{tag}: {json.dumps(out[tag])}")
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serving benchmark: continuous batching vs sequential solves")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--max-active", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    args = ap.parse_args(argv)
    print(json.dumps(serving_benchmark(args.requests, n_streams=args.streams, max_active=args.max_active,
                                       budget_gb=args.budget_gb)), flush=True)


if __name__ == "__main__":
    main()
