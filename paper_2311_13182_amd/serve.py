"""Serving loop: a persistent scheduler that runs forward and forward+backward
simulations of many requests on one GPU with continuous batching.

* Admission by device-memory footprint: a request is admitted when its
  footprint (exactly the device buffers its pipeline allocates) fits the part
  of the budget that active requests and idle cached meshes leave free (FIFO
  order; idle cache entries are evicted to make room; a request larger than
  the whole budget is rejected).
* Continuous batching: at every scheduling tick the requests admitted since
  the last one form a batch (or several of at most max_batch requests).
  Their per-request stages (mesh upload, BVH build, trace, path refinement)
  are enqueued on one HIP stream, then ONE batched IF-synthesis launch covers
  the synthesis blocks of all of them (sbr_synth_if_batched), and the
  forward+backward ones share ONE batched adjoint launch
  (sbr_backward_batched).  Consecutive batches go to different streams, so a
  batch admitted while others run overlaps them on the device, and the host
  prepares one batch while the device runs the previous one.
* BVHs and meshes stay resident for the life of a request, and repeated
  meshes (same vertices, faces and materials) reuse a cached device copy: a
  request that hits the cache waits (on the device) for the event that ends
  the copy's upload and build on the stream that made it.
* An optional per-request timeout fails a request that stays active too long
  and releases what it holds.
* Each request's launch shapes depend only on its own sizes, so its forward
  result is bit-identical alone and in the mix (the backward differs only in
  the order of floating-point atomics).

The scheduler is independent of the device: `Scheduler` drives any object
with the executor interface (`footprint`, `launch`, `poll`, `collect`,
`release`, optionally `launch_batch`, `resident_bytes` and `evict_idle`),
which the tests replace with a CPU fake.
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
    hits: Optional[Dict[str, np.ndarray]] = None   # tri / flags when the executor returns them

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Scheduler:
    """Admission + continuous batching over an executor.  Thread-safe submit."""

    def __init__(self, executor, budget_bytes: int, max_active: int = 16, clock=time.perf_counter,
                 request_timeout: Optional[float] = None, max_batch: Optional[int] = None,
                 collect_workers: int = 0):
        """request_timeout: seconds a request may stay active (admitted, not
        finished) before it is failed and its resources released; None waits
        for ever.  max_batch: most requests per batched launch; the requests
        admitted in one tick are launched in groups of at most that many
        (None: one group), so the host prepares one group while the device
        runs the previous one.  collect_workers: threads that copy finished
        requests' results out of the executor's host buffers (0: the
        scheduler thread copies them itself).  The copy into fresh client
        memory costs about as much host time as a launch, and NumPy drops the
        GIL while it runs, so with workers it overlaps the next launches; the
        scheduler thread still releases each request and settles its budget
        and future once its copy is done."""
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.request_timeout = request_timeout
        self.max_batch = max_batch
        self.batch_fallbacks: List[str] = []   # errors of batches relaunched one request at a time
        self.clock = clock
        self.t0 = clock()
        self._pending: Deque = collections.deque()
        self._active: List = []
        self._used = 0
        self._admitting = 0          # requests taken off the queue, not yet in _active or finished
        self._footprints: Dict[int, int] = {}
        self._lock = threading.Lock()
        self._stop = threading.Event()
        self._thread: Optional[threading.Thread] = None
        self.log: List[Result] = []
        self._collector = (concurrent.futures.ThreadPoolExecutor(int(collect_workers),
                                                                thread_name_prefix="sbr-collect")
                           if collect_workers > 0 else None)

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
            req, fut, h, fp, t_admit, cf = item
            if cf is not None:   # results being copied out by a worker
                if cf.done():
                    err = cf.exception()
                    self._finish(req, fut, h, fp, t_admit, None if err is not None else cf.result(), err)
                    progressed = True
                else:
                    still.append(item)
                continue
            try:
                done = self.ex.poll(h)
            except Exception as e:   # device-side failure of this request only
                self._finish(req, fut, h, fp, t_admit, None, e)
                progressed = True
                continue
            if not done and self.request_timeout is not None and self.now() - t_admit > self.request_timeout:
                self._finish(req, fut, h, fp, t_admit, None,
                             TimeoutError(f"request {req.rid} active for more than {self.request_timeout} s"))
                progressed = True
                continue
            if done and self._collector is not None:
                still.append((req, fut, h, fp, t_admit, self._collector.submit(self.ex.collect, h)))
                progressed = True
            elif done:
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
        admitted = []
        n_active = len(self._active)
        while True:
            with self._lock:
                if not self._pending or self._pending[0][0].arrival > now:
                    break
                req, fut = self._pending[0]
                fp = self._footprints.get(req.rid)
                if fp is None:
                    try:
                        fp = self._footprints[req.rid] = int(self.ex.footprint(req))
                    except Exception as e:   # a request that cannot be sized fails alone
                        self._pending.popleft()
                        res = Result(req.rid, "failed", t_arrival=req.arrival, t_done=now,
                                     error=f"footprint: {e!r}")
                        self.log.append(res)
                        fut.set_result(res)
                        progressed = True
                        continue
                if fp > self.budget:
                    self._pending.popleft()
                    res = Result(req.rid, "rejected", t_arrival=req.arrival, t_done=now, footprint=fp,
                                 error=f"footprint {fp} B exceeds the budget {self.budget} B")
                    self.log.append(res)
                    fut.set_result(res)
                    progressed = True
                    continue
                if n_active + len(admitted) >= self.max_active:
                    break
                if self._used + fp + self.resident_bytes() > self.budget:
                    # idle cached meshes give way to requests
                    self._evict(self._used + fp + self.resident_bytes() - self.budget)
                    if self._used + fp + self.resident_bytes() > self.budget:
                        break
                self._pending.popleft()
                self._admitting += 1
            self._used += fp
            admitted.append((req, fut, fp))
        if admitted:
            step = self.max_batch or len(admitted)
            try:
                for g in range(0, len(admitted), step):
                    self._launch(admitted[g:g + step])
            finally:
                with self._lock:
                    self._admitting -= len(admitted)
            progressed = True
        return progressed

    def resident_bytes(self) -> int:
        """Device bytes the executor holds outside active requests (idle cache)."""
        f = getattr(self.ex, "resident_bytes", None)
        return int(f()) if f is not None else 0

    def _evict(self, nbytes: int):
        f = getattr(self.ex, "evict_idle", None)
        if f is not None:
            f(int(nbytes))

    def _fail_launch(self, req, fut, fp, t_admit, e):
        self._used -= fp
        res = Result(req.rid, "failed", t_arrival=req.arrival, t_admit=t_admit, t_done=self.now(),
                     footprint=fp, error=repr(e))
        self.log.append(res)
        fut.set_result(res)

    def _launch(self, admitted):
        """One batch for the executor (or one launch per request without
        launch_batch, or when the batch as a whole fails: then each request
        is launched alone so that a bad request fails only itself)."""
        t_admit = self.now()
        batch = getattr(self.ex, "launch_batch", None)
        if batch is not None and len(admitted) > 1:
            try:
                hs = batch([a[0] for a in admitted])
                for (req, fut, fp), h in zip(admitted, hs):
                    self._active.append((req, fut, h, fp, t_admit, None))
                return
            except Exception as e:   # fall back to single launches below
                self.batch_fallbacks.append(repr(e))
        for req, fut, fp in admitted:
            try:
                h = self.ex.launch(req)
            except Exception as e:
                self._fail_launch(req, fut, fp, t_admit, e)
                continue
            self._active.append((req, fut, h, fp, t_admit, None))

    def _finish(self, req, fut, h, fp, t_admit, out, err):
        try:
            self.ex.release(h)
        finally:
            self._used -= fp
        if err is None:
            res = Result(req.rid, "ok", cube=out.get("cube"), grad=out.get("grad"), n_paths=out.get("n_paths", -1),
                         t_arrival=req.arrival, t_admit=t_admit, t_done=self.now(), footprint=fp,
                         hits={k: out[k] for k in ("tri", "flags") if k in out} or None)
        else:
            res = Result(req.rid, "failed", t_arrival=req.arrival, t_admit=t_admit, t_done=self.now(),
                         footprint=fp, error=repr(err))
        self.log.append(res)
        fut.set_result(res)

    def idle(self) -> bool:
        with self._lock:
            return not self._pending and not self._admitting and not self._active

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
        # anything left is failed explicitly (never silently dropped), after
        # any copy of its results still reading the executor's buffers
        for req, fut, h, fp, t_admit, cf in self._active:
            if cf is not None:
                concurrent.futures.wait([cf])
            self._finish(req, fut, h, fp, t_admit, None, RuntimeError("scheduler stopped"))
        self._active = []
        if self._collector is not None:
            self._collector.shutdown(wait=True)
            self._collector = None
        with self._lock:
            while self._pending:
                req, fut = self._pending.popleft()
                res = Result(req.rid, "failed", t_arrival=req.arrival, t_done=self.now(), error="scheduler stopped")
                self.log.append(res)
                fut.set_result(res)


# --------------------------------------------------------------------------- GPU executor
def _dev_bytes(n: int) -> int:
    """Most bytes the caching allocator books for an n-byte tensor: blocks of
    512 bytes, and a block of its large pool (over 1 MiB) keeps the rest of
    the segment it comes from when that rest is 1 MiB or less."""
    r = (int(n) + 511) // 512 * 512
    return r if r <= (1 << 20) else r + (1 << 20)


def mesh_bytes(scene: S.Scene) -> int:
    """Device bytes of a resident mesh and its BVH (the cached part of a request)."""
    from . import sbr as B
    b = _dev_bytes(scene.nv * 12) + _dev_bytes(scene.nf * 12)
    if scene.mat_id is not None:
        b += _dev_bytes(scene.nf * 2)
    return b + _dev_bytes(max(1, B.sbr_bvh_bytes(scene.nf)))


def request_footprint(scene: S.Scene, backward: bool) -> int:
    """Device bytes a request's pipeline allocates while it is active: mesh
    and BVH (counted even when a cached copy is reused), the Simulator's
    scratch sized for the stages it runs, hit records, counters, the loss
    partials, the IF cube and path count; for forward+backward also the
    target cube, dL/dIF, the loss and dL/dverts; plus the request's share of
    the batch table."""
    from . import sbr as B
    g, rd, ch = scene.grid, scene.radar, scene.chirp
    V, C, Sn, R, K = rd.n_virtual, ch.n_chirps, ch.n_samples, g.n_rays, g.max_bounces
    cube = _dev_bytes(V * C * Sn * 8)
    b = mesh_bytes(scene)
    b += _dev_bytes(B.simulator_scratch_bytes(scene, backward=backward, cube=False))
    b += 4 * _dev_bytes(4 * R * K) + _dev_bytes(R * K)        # tri, t, u, v, flags
    b += _dev_bytes(24) + _dev_bytes(8192)                    # counters, loss partials
    b += cube + _dev_bytes(4)                                 # IF cube, path count
    if backward:
        b += 2 * cube + _dev_bytes(4) + _dev_bytes(scene.nv * 12)   # target, dL/dIF, loss, dL/dverts
    return int(b + _dev_bytes(B.sbr_batch_table_bytes(1)))


def _mesh_key(scene: S.Scene) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(scene.verts).tobytes())
    h.update(np.ascontiguousarray(scene.faces).tobytes())
    if scene.mat_id is not None:
        h.update(np.ascontiguousarray(scene.mat_id).astype(np.int64).tobytes())
    h.update(repr([tuple(float(x) for x in m) for m in scene.materials]).encode())
    return h.hexdigest()


@dataclasses.dataclass
class _MeshEntry:
    mesh: Any            # DeviceMesh
    bvh: Any             # uint8 tensor
    ready: Any           # torch.cuda.Event recorded after upload + build
    nbytes: int
    refs: int = 0        # active requests using it


class GPUExecutor:
    """Runs batches of requests on `n_streams` HIP streams in turn (one stream
    per batch); meshes and BVHs are cached by content, reference-counted."""

    def __init__(self, device="cuda", n_streams: int = 4, cache_meshes: int = 8, extra_flags=None,
                 return_hits: bool = False):
        """extra_flags: None, or a callable request -> None or uint8 [K, R]
        hit flags to OR into the request's traced flags before synthesis (rays
        a caller wants dropped, e.g. those another implementation flags when
        results are compared record by record).  return_hits: results also
        carry the hit ids and flags the synthesis used ("tri", "flags")."""
        import torch
        self.torch = torch
        self.extra_flags = extra_flags
        self.return_hits = return_hits
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]  # default priority
        self.next = 0
        self.cache: "collections.OrderedDict[str, _MeshEntry]" = collections.OrderedDict()
        self.cache_meshes = cache_meshes
        self.batch_sizes: List[int] = []   # requests per launched batch, in launch order

    def footprint(self, req: Request) -> int:
        return request_footprint(req.scene, req.backward)

    # ---- mesh cache
    def resident_bytes(self) -> int:
        """Bytes of cached meshes and BVHs that no active request uses."""
        return sum(e.nbytes for e in self.cache.values() if e.refs == 0)

    def evict_idle(self, nbytes: int) -> int:
        """Drop idle cache entries, least recently used first, until `nbytes`
        are freed (or none is idle); returns the bytes freed."""
        freed = 0
        for key in list(self.cache.keys()):
            if freed >= nbytes:
                break
            e = self.cache[key]
            if e.refs == 0:
                del self.cache[key]
                freed += e.nbytes
        return freed

    def _trim(self):
        idle = [k for k, e in self.cache.items() if e.refs == 0]
        while len(self.cache) > self.cache_meshes and idle:
            del self.cache[idle.pop(0)]

    def _mesh_for(self, req: Request, st):
        """(key, entry) of the request's mesh on stream st: a cached copy (st
        waits for its ready event) or a fresh upload + BVH build on st."""
        from .sbr import DeviceMesh, sbr_build_bvh, sbr_bvh_bytes, sbr_scratch_bytes
        from . import _lib as L
        torch = self.torch
        key = _mesh_key(req.scene)
        e = self.cache.get(key)
        if e is not None:
            self.cache.move_to_end(key)
            st.wait_event(e.ready)
            for t in (e.mesh.verts, e.mesh.faces, e.bvh):
                t.record_stream(st)
            if e.mesh.mat_id is not None:
                e.mesh.mat_id.record_stream(st)
        else:
            mesh = DeviceMesh.from_scene(req.scene, self.device, non_blocking=True)
            bvh = torch.empty(max(1, sbr_bvh_bytes(mesh.nf)), dtype=torch.uint8, device=self.device)
            if mesh.nf > 0:
                bs = torch.empty(max(1, sbr_scratch_bytes(L.SBR_OP_BUILD_BVH, mesh)), dtype=torch.uint8,
                                 device=self.device)
                sbr_build_bvh(mesh, bvh, 0, bs)
            ready = torch.cuda.Event()
            ready.record(st)
            e = _MeshEntry(mesh, bvh, ready, mesh_bytes(req.scene))
            self.cache[key] = e
        e.refs += 1
        return key, e

    # ---- launches
    def launch(self, req: Request):
        return self.launch_batch([req])[0]

    def launch_batch(self, reqs: List[Request]):
        """Enqueue the requests' pipelines on the next stream: per request
        mesh (cached or uploaded + built) and trace, then one batched
        synthesis over all of them and one batched adjoint over the
        forward+backward ones; results are copied to pinned host buffers
        behind one event.  Returns one handle per request."""
        torch = self.torch
        from .sbr import Simulator, sbr_backward_batched, sbr_batch_table_bytes, sbr_synth_if_batched
        st = self.streams[self.next % len(self.streams)]
        self.next += 1
        hs: List[Dict[str, Any]] = [dict(stream=st) for _ in reqs]
        keys: List[str] = []
        try:
            with torch.cuda.stream(st):
                sims = []
                for req, h in zip(reqs, hs):
                    key, e = self._mesh_for(req, st)
                    keys.append(key)
                    h["mesh_key"] = key
                    sim = Simulator(req.scene, self.device, mesh=e.mesh, bvh=e.bvh, backward=req.backward,
                                    cube=False)
                    sim.trace()
                    extra = self.extra_flags(req) if self.extra_flags is not None else None
                    if extra is not None:
                        fl = torch.from_numpy(np.ascontiguousarray(extra, dtype=np.uint8)).pin_memory()
                        h["flag_staging"] = fl
                        sim.hits.flags.bitwise_or_(fl.to(self.device, non_blocking=True).view_as(sim.hits.flags))
                    sims.append(sim)
                    h["sim"] = sim
                table = torch.empty(max(1, sbr_batch_table_bytes(len(reqs))), dtype=torch.uint8,
                                    device=self.device)
                cubes = [torch.empty((s.V, s.C, s.S, 2), dtype=torch.float32, device=self.device) for s in sims]
                sbr_synth_if_batched([(s.mesh, s.scene.radar, s.scene.grid, s.hits, s.scene.chirp, s.flags, c,
                                       s.scratch) for s, c in zip(sims, cubes)], table)
                for h, s, c in zip(hs, sims, cubes):
                    h["cube"] = c
                    # the synthesis leaves the path count in the scratch buffer
                    h["n_paths_dev"] = s.scratch[:4].view(torch.int32).clone()
                bw = [i for i, r in enumerate(reqs) if r.backward]
                if bw:
                    items = []
                    for i in bw:
                        s, h = sims[i], hs[i]
                        th = torch.from_numpy(np.ascontiguousarray(reqs[i].target, dtype=np.complex64)).pin_memory()
                        h["target_staging"] = th
                        tgt = th.to(self.device, non_blocking=True)
                        grad_if, _ = s.loss_grad(h["cube"], tgt)
                        gv = torch.zeros((s.mesh.nv, 3), dtype=torch.float32, device=self.device)
                        h["grad"] = gv
                        items.append((s.mesh, s.scene.radar, s.scene.grid, s.hits, s.scene.chirp, s.flags, grad_if,
                                      gv, s.scratch))
                    sbr_backward_batched(items, table)
                # one pinned host buffer per batch for every request's cube,
                # gradient and path count (instead of two or three pinned
                # allocations per request), sliced per request
                def span(n):   # slice lengths rounded up to 64 floats (256 B)
                    return (n + 63) // 64 * 64
                n_f32 = sum(span(h["cube"].numel()) + (span(h["grad"].numel()) if "grad" in h else 0) for h in hs)
                host_f32 = torch.empty(max(1, n_f32), dtype=torch.float32, pin_memory=True)
                host_i32 = torch.empty(len(hs), dtype=torch.int32, pin_memory=True)
                off = 0
                for i, h in enumerate(hs):
                    n_c = h["cube"].numel()
                    h["cube_host"] = host_f32[off:off + n_c].view(h["cube"].shape)
                    off += span(n_c)
                    h["cube_host"].copy_(h["cube"], non_blocking=True)
                    h["np_host"] = host_i32[i:i + 1]
                    h["np_host"].copy_(h["n_paths_dev"], non_blocking=True)
                    if "grad" in h:
                        n_g = h["grad"].numel()
                        h["grad_host"] = host_f32[off:off + n_g].view(h["grad"].shape)
                        off += span(n_g)
                        h["grad_host"].copy_(h["grad"], non_blocking=True)
                    if self.return_hits:
                        for name in ("tri", "flags"):
                            src = getattr(h["sim"].hits, name)
                            h[name + "_host"] = torch.empty(src.shape, dtype=src.dtype, pin_memory=True)
                            h[name + "_host"].copy_(src, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(st)
                for h in hs:
                    h["event"] = ev
                    h["table"] = table
        except Exception:
            for key in keys:
                self._unref(key)
            raise
        self._trim()
        self.batch_sizes.append(len(reqs))
        return hs

    def _unref(self, key):
        e = self.cache.get(key)
        if e is not None:
            e.refs -= 1

    def poll(self, h) -> bool:
        return h["event"].query()

    def collect(self, h) -> Dict[str, Any]:
        h["event"].synchronize()
        res = {"cube": h["cube_host"].numpy().view(np.complex64).reshape(h["cube"].shape[:-1]).copy(),
               "n_paths": int(h["np_host"][0])}
        if "grad_host" in h:
            res["grad"] = h["grad_host"].numpy().copy()
        for name in ("tri", "flags"):
            if name + "_host" in h:
                res[name] = h[name + "_host"].numpy().copy()
        return res

    def release(self, h):
        key = h.get("mesh_key")
        if key is not None:
            self._unref(key)
        h.clear()
        self._trim()


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
                          t_arrival=req.arrival, t_admit=ta, t_done=time.perf_counter() - t0,
                          hits={k: r[k] for k in ("tri", "flags") if k in r} or None))
    return out


def summarize(results: List[Result], wall: float) -> Dict[str, float]:
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    return {"requests": len(results), "ok": len(ok), "wall_s": wall, "throughput_rps": len(ok) / wall,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3), "p99_latency_ms": float(np.percentile(lat, 99) * 1e3)}


def _batch_stats(sizes: List[int]) -> Dict[str, float]:
    return {"launches": len(sizes), "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
            "max_batch": int(max(sizes)) if sizes else 0}


def serving_benchmark(n: int = 512, seed: int = 5, budget_gb: float = 64.0, n_streams: int = 4,
                      max_active: int = 16, grids=(256, 512, 1024, 2048), nf_range=(1000, 200000),
                      phases=(("main", 1.25), ("low", 0.5)), quiet: bool = False, burst: int = 128,
                      collect_workers: int = 2):
    """Sequential FIFO solves vs the continuous-batching server on the same
    Poisson request stream (QPS = 1.25 x the measured sequential rate), with
    the server's batch sizes; then a burst of `burst` small forward requests
    that all arrive at once (256^2 rays, 1k-20k triangles, 32 chirps), where
    admitted requests share batched launches of up to 16.  The server copies
    results out on `collect_workers` threads."""
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
    out = {"mu_seq_rps": mu, "n_backward": sum(r.backward for r in reqs), "collect_workers": collect_workers}
    for tag, factor in phases:
        qps = factor * mu
        rng = np.random.default_rng(seed + 1)
        arr = np.cumsum(rng.exponential(1.0 / qps, size=n))
        timed = [Request(r.rid, r.scene, r.backward, r.target, float(a)) for r, a in zip(reqs, arr)]
        seq = run_sequential(ex, timed)
        seq_w = max(r.t_done for r in seq)
        sch = Scheduler(ex, int(budget_gb * (1 << 30)), max_active=max_active, collect_workers=collect_workers)
        futs = [sch.submit(r) for r in timed]
        ex.batch_sizes.clear()
        sch.t0 = time.perf_counter()
        sch.start()
        res = [f.result() for f in futs]
        sch.stop()
        srv_w = max(r.t_done for r in res)
        out[tag] = {"qps": qps, "sequential": summarize(seq, seq_w),
                    "server": {**summarize(res, srv_w), **_batch_stats(ex.batch_sizes),
                               "batch_fallbacks": len(sch.batch_fallbacks)}}
        if sch.batch_fallbacks:
            say(f"{tag}: batches relaunched one request at a time: {sch.batch_fallbacks[:3]}")
        say(f"{tag}: {json.dumps(out[tag])}")
    if burst > 0:
        # all requests admitted at once (max_active = burst), launched in
        # groups of 16; three repetitions of each mode, the median reported
        small = S.serving_requests(n=burst, qps=1.0, seed=seed + 2, grids=(256,), nf_range=(1000, 20000),
                                   chirps=(32,))
        reqs_b = [Request(r.rid, r.scene, False, None, 0.0) for r in small]
        h = ex.launch(reqs_b[0])     # warm the shapes of this mix (untimed)
        ex.collect(h)
        ex.release(h)
        runs = {"sequential": [], "server": []}
        for _ in range(3):
            seq = run_sequential(ex, reqs_b)
            runs["sequential"].append(summarize(seq, max(r.t_done for r in seq)))
            sch = Scheduler(ex, int(budget_gb * (1 << 30)), max_active=burst, max_batch=16,
                            collect_workers=collect_workers)
            ex.batch_sizes.clear()
            sch.t0 = time.perf_counter()   # every request arrives at time 0
            futs = [sch.submit(Request(r.rid, r.scene, False, None, 1e-9)) for r in reqs_b]
            sch.start()
            res = [f.result() for f in futs]
            sch.stop()
            runs["server"].append({**summarize(res, max(r.t_done for r in res)), **_batch_stats(ex.batch_sizes)})
        med = {k: sorted(v, key=lambda r: r["throughput_rps"])[1] for k, v in runs.items()}
        out["burst"] = {"requests": burst, "repetitions": 3, **med,
                        "server_launches_per_repetition": [r["launches"] for r in runs["server"]]}
        say(f"burst: {json.dumps(out['burst'])}")
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serving benchmark: continuous batching vs sequential solves")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--max-active", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--collect-workers", type=int, default=2)
    args = ap.parse_args(argv)
    print(json.dumps(serving_benchmark(args.requests, n_streams=args.streams, max_active=args.max_active,
                                       budget_gb=args.budget_gb, collect_workers=args.collect_workers)),
          flush=True)


if __name__ == "__main__":
    main()
