"""Python binding of libsbr with the C ABI's names.

PyTorch provides device memory and the HIP stream; every step of the
simulation runs in libsbr's HIP kernels.  Functions enqueue on
`torch.cuda.current_stream()` and return without synchronising.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from . import scenes as S

EXPORTS = L.EXPORTS


def _lib():
    return L.load()


def _p(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ct.c_void_p(t.data_ptr())


def _buf(t: Optional[torch.Tensor], dtype, n: int, name: str, optional: bool = False):
    """Pointer to a buffer the C ABI writes or reads without knowing its size,
    after the checks it cannot make itself: dtype, contiguity, at least `n`
    elements, device memory.  Raises ValueError instead of letting a kernel
    run past the end of a buffer."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, {n} needed")
    if not t.is_cuda:
        raise ValueError(f"{name} must be in device memory")
    return ct.c_void_p(t.data_ptr())


def _check_hits(h: "Hits", K: int, R: int):
    for f, dt in (("tri", torch.int32), ("t", torch.float32), ("u", torch.float32), ("v", torch.float32),
                  ("flags", torch.uint8)):
        _buf(getattr(h, f), dt, K * R, f"hits.{f}")


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


# ----------------------------------------------------------------- structs
def radar_struct(r: S.Radar) -> L.sbr_radar:
    s = L.sbr_radar()
    if r.n_tx > L.SBR_MAX_TX or r.n_rx > L.SBR_MAX_RX:
        raise ValueError("too many TX / RX antennas")
    for i in range(3):
        s.origin[i] = float(r.origin[i])
        s.velocity[i] = float(r.vel[i])
    s.attenuation = float(getattr(r, "atten", 0.0))
    s.tx_gain_exp = float(getattr(r, "n_tx_gain", 0.0))
    s.rx_gain_exp = float(getattr(r, "n_rx_gain", 0.0))
    rot = np.asarray(r.rot, dtype=np.float64).reshape(-1)
    for i in range(9):
        s.rot[i] = float(rot[i])
    s.n_tx, s.n_rx = r.n_tx, r.n_rx
    for t in range(r.n_tx):
        for j in range(3):
            s.tx[t][j] = float(r.tx[t][j])
    for m in range(r.n_rx):
        for j in range(3):
            s.rx[m][j] = float(r.rx[m][j])
    return s


def chirp_struct(c: S.Chirp) -> L.sbr_chirp:
    return L.sbr_chirp(c.fc, c.slope, c.fs, c.t_chirp, c.n_samples, c.n_chirps)


def rays_struct(g: S.Grid) -> L.sbr_rays:
    seed = getattr(g, "jitter_seed", None)
    opts = (L.SBR_RAYS_SHADOW if getattr(g, "shadow", False) else 0) | (L.SBR_RAYS_JITTER if seed is not None else 0)
    return L.sbr_rays(g.nx, g.ny, g.tan_hx, g.tan_hy, g.max_bounces, opts, g.t_min, (seed or 0) & 0xFFFFFFFF,
                      ((seed or 0) >> 32) & 0xFFFFFFFF)


def materials_struct(mats: Sequence[Tuple[int, float, float]]):
    n = len(mats)
    if n == 0:
        return None, 0
    arr = (L.sbr_material * n)()
    for i, (mode, er, sg) in enumerate(mats):
        arr[i].mode, arr[i].eps_r, arr[i].sigma = int(mode), float(er), float(sg)
    return arr, n


class DeviceMesh:
    """Mesh resident on the device: verts float32 [nv,3], faces int32 [nf,3],
    optional per-face material ids (uint16 stored as int16)."""

    def __init__(self, verts, faces, mat_id=None, materials=(), device="cuda"):
        self.verts = torch.as_tensor(np.ascontiguousarray(verts, np.float32) if isinstance(verts, np.ndarray)
                                     else verts, dtype=torch.float32, device=device).contiguous()
        self.faces = torch.as_tensor(np.ascontiguousarray(faces, np.int32) if isinstance(faces, np.ndarray)
                                     else faces, dtype=torch.int32, device=device).contiguous()
        self.mat_id = None
        if mat_id is not None:
            self.mat_id = torch.as_tensor(np.asarray(mat_id).astype(np.int16), device=device).contiguous()
        self.materials = list(materials)

    @property
    def nv(self):
        return int(self.verts.shape[0])

    @property
    def nf(self):
        return int(self.faces.shape[0])

    def struct(self) -> L.sbr_mesh:
        return L.sbr_mesh(self.verts.data_ptr(), self.nv, self.faces.data_ptr(), self.nf,
                          self.mat_id.data_ptr() if self.mat_id is not None else None)

    @classmethod
    def from_scene(cls, sc: S.Scene, device="cuda", non_blocking: bool = False):
        if not non_blocking:
            return cls(sc.verts, sc.faces, sc.mat_id, sc.materials, device)
        # one pinned staging buffer for vertices, faces and material ids
        # (one pinned allocation per mesh instead of one per array), then
        # asynchronous copies on the current stream into the mesh's own
        # device tensors; the staging buffer lives as long as the mesh
        self = cls.__new__(cls)
        parts = [np.ascontiguousarray(sc.verts, np.float32).reshape(-1).view(np.uint8),
                 np.ascontiguousarray(sc.faces, np.int32).reshape(-1).view(np.uint8)]
        if sc.mat_id is not None:
            parts.append(np.asarray(sc.mat_id).astype(np.int16).reshape(-1).view(np.uint8))
        offs = np.cumsum([0] + [(len(x) + 255) // 256 * 256 for x in parts])
        st = torch.empty(int(offs[-1]), dtype=torch.uint8, pin_memory=True)
        host = st.numpy()
        for x, o in zip(parts, offs):
            host[o:o + len(x)] = x
        def up(i, dt, shape):
            return st[int(offs[i]):int(offs[i]) + len(parts[i])].view(dt).view(shape).to(device, non_blocking=True)
        self.verts = up(0, torch.float32, (-1, 3))
        self.faces = up(1, torch.int32, (-1, 3))
        self.mat_id = up(2, torch.int16, (-1,)) if sc.mat_id is not None else None
        self._staging = [st]
        self.materials = list(sc.materials)
        return self


@dataclasses.dataclass
class Hits:
    tri: torch.Tensor      # int32 [K, R]
    t: torch.Tensor        # float32 [K, R]
    u: torch.Tensor
    v: torch.Tensor
    flags: torch.Tensor    # uint8 [K, R]

    @classmethod
    def empty(cls, K: int, R: int, device="cuda"):
        return cls(torch.empty((K, R), dtype=torch.int32, device=device),
                   torch.empty((K, R), dtype=torch.float32, device=device),
                   torch.empty((K, R), dtype=torch.float32, device=device),
                   torch.empty((K, R), dtype=torch.float32, device=device),
                   torch.empty((K, R), dtype=torch.uint8, device=device))

    def struct(self) -> L.sbr_hits:
        return L.sbr_hits(self.tri.data_ptr(), self.t.data_ptr(), self.u.data_ptr(), self.v.data_ptr(),
                          self.flags.data_ptr())


# ----------------------------------------------------------------- entry points
def sbr_bvh_bytes(nf: int) -> int:
    return int(_lib().sbr_bvh_bytes(int(nf)))


def sbr_scratch_bytes(op: int, mesh: Optional[DeviceMesh] = None, rays: Optional[S.Grid] = None,
                      radar: Optional[S.Radar] = None, chirp: Optional[S.Chirp] = None) -> int:
    m = mesh.struct() if mesh is not None else None
    g = rays_struct(rays) if rays is not None else None
    r = radar_struct(radar) if radar is not None else None
    c = chirp_struct(chirp) if chirp is not None else None
    return int(_lib().sbr_scratch_bytes(int(op), ct.byref(m) if m else None, ct.byref(g) if g else None,
                                        ct.byref(r) if r else None, ct.byref(c) if c else None))


def sbr_build_bvh(mesh: DeviceMesh, bvh: torch.Tensor, mode: int = 0, scratch: Optional[torch.Tensor] = None):
    m = mesh.struct()
    L.check(_lib().sbr_build_bvh(ct.byref(m), _p(bvh), bvh.numel() * bvh.element_size(), int(mode), _p(scratch),
                                 0 if scratch is None else scratch.numel() * scratch.element_size(), _stream()))


def sbr_trace(mesh: DeviceMesh, bvh: Optional[torch.Tensor], radar: S.Radar, rays: S.Grid, hits: Hits,
              counters: Optional[torch.Tensor] = None):
    _check_hits(hits, rays.max_bounces, rays.nx * rays.ny)
    cnt = _buf(counters, torch.int64, 3, "counters", optional=True)
    m, r, g, h = mesh.struct(), radar_struct(radar), rays_struct(rays), hits.struct()
    L.check(_lib().sbr_trace(ct.byref(m), _p(bvh), ct.byref(r), ct.byref(g), ct.byref(h), cnt, _stream()))


def sbr_synth_if(mesh: DeviceMesh, radar: S.Radar, rays: S.Grid, hits: Hits, chirp: S.Chirp, flags: int,
                 if_cube: torch.Tensor, scratch: torch.Tensor):
    out = _buf(if_cube, torch.float32, 2 * radar.n_virtual * chirp.n_chirps * chirp.n_samples, "if_cube")
    _check_hits(hits, rays.max_bounces, rays.nx * rays.ny)
    sp = _buf(scratch, torch.uint8, 0, "scratch")
    m, r, g, h, c = mesh.struct(), radar_struct(radar), rays_struct(rays), hits.struct(), chirp_struct(chirp)
    mats, nm = materials_struct(mesh.materials)
    L.check(_lib().sbr_synth_if(ct.byref(m), mats, nm, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c),
                                int(flags), out, sp, scratch.numel() * scratch.element_size(), _stream()))


def sbr_radar_cube_2d_bytes(vx: int, vy: int, C: int, Sn: int, n_ax: int, n_ay: int) -> int:
    return int(_lib().sbr_radar_cube_2d_bytes(vx, vy, C, Sn, n_ax, n_ay))


def sbr_radar_cube_2d(x: torch.Tensor, vx: int, vy: int, C: int, Sn: int, n_ax: int, n_ay: int, window: int,
                      direction: int, out: torch.Tensor, scratch: torch.Tensor):
    nv, na = vx * vy * C * Sn * 2, n_ax * n_ay * C * Sn * 2
    xi = _buf(x, torch.float32, nv if direction == 0 else na, "x")
    xo = _buf(out, torch.float32, na if direction == 0 else nv, "out")
    L.check(_lib().sbr_radar_cube_2d(xi, vx, vy, C, Sn, n_ax, n_ay, window, direction, xo,
                                     _buf(scratch, torch.uint8, 0, "scratch"),
                                     scratch.numel() * scratch.element_size(), _stream()))


def sbr_angle_peaks(X: torch.Tensor, n_ax: int, n_ay: int, C: int, Sn: int, det: torch.Tensor, n_det: torch.Tensor,
                    rel: float = 0.1, max_points: int = 65536):
    """Angle peaks of detected cells of a radar cube [n_ay*n_ax, C, S] (complex
    or [.., 2] float).  Returns (points [max_points, 4] int32, count [1])."""
    xf = (torch.view_as_real(X) if X.is_complex() else X).contiguous()
    need = int(_lib().sbr_angle_peaks_bytes(int(det.shape[0]), n_ax, n_ay))
    scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=xf.device)
    pts = torch.empty((max_points, 4), dtype=torch.int32, device=xf.device)
    n = torch.zeros(1, dtype=torch.int32, device=xf.device)
    xp = _buf(xf, torch.float32, 2 * n_ax * n_ay * C * Sn, "X")
    dp = _buf(det, torch.int32, 4 * int(det.shape[0]), "det")
    L.check(_lib().sbr_angle_peaks(xp, n_ax, n_ay, C, Sn, dp, _buf(n_det, torch.int32, 1, "n_det"),
                                   int(det.shape[0]), ct.c_float(rel), _p(pts), max_points, _p(n), _p(scratch), need,
                                   _stream()))
    return pts, n


def sbr_cloud(points: torch.Tensor, n_points: torch.Tensor, radar: S.Radar, chirp: S.Chirp, n_ax: int, n_ay: int,
              out: torch.Tensor):
    r, c = radar_struct(radar), chirp_struct(chirp)
    mp = int(points.shape[0])
    L.check(_lib().sbr_cloud(_buf(points, torch.int32, 4 * mp, "points"), _buf(n_points, torch.int32, 1, "n_points"),
                             mp, ct.byref(r), ct.byref(c), n_ax, n_ay, _buf(out, torch.float32, 4 * mp, "out"),
                             _stream()))


def sbr_radar_cube(x: torch.Tensor, V: int, C: int, Sn: int, n_angle: int, window: int, direction: int,
                   out: torch.Tensor, scratch: torch.Tensor):
    nv, na = V * C * Sn * 2, n_angle * C * Sn * 2
    xi = _buf(x, torch.float32, nv if direction == 0 else na, "x")
    xo = _buf(out, torch.float32, na if direction == 0 else nv, "out")
    L.check(_lib().sbr_radar_cube(xi, V, C, Sn, n_angle, window, direction, xo, _buf(scratch, torch.uint8, 0, "scratch"),
                                  scratch.numel() * scratch.element_size(), _stream()))


def sbr_radar_cube_noalloc(x: torch.Tensor, V: int, C: int, Sn: int, n_angle: int, window: int, direction: int,
                           out: torch.Tensor):
    """sbr_radar_cube with the library's own static staging buffers (no scratch)."""
    nv, na = V * C * Sn * 2, n_angle * C * Sn * 2
    xi = _buf(x, torch.float32, nv if direction == 0 else na, "x")
    xo = _buf(out, torch.float32, na if direction == 0 else nv, "out")
    L.check(_lib().sbr_radar_cube_noalloc(xi, V, C, Sn, n_angle, window, direction, xo, _stream()))


def sbr_cfar(cube: torch.Tensor, Na: int, C: int, Sn: int, guard: int, train: int, pfa: float,
             points: torch.Tensor, ratio: Optional[torch.Tensor], n_points: torch.Tensor, scratch: torch.Tensor):
    mp = int(points.shape[0])
    L.check(_lib().sbr_cfar(_buf(cube, torch.float32, 2 * Na * C * Sn, "cube"), Na, C, Sn, guard, train, float(pfa),
                            _buf(points, torch.int32, 4 * mp, "points"),
                            _buf(ratio, torch.float32, mp, "ratio", optional=True), mp,
                            _buf(n_points, torch.int32, 1, "n_points"), _buf(scratch, torch.uint8, 0, "scratch"),
                            scratch.numel() * scratch.element_size(), _stream()))


def _param_grads(mesh: DeviceMesh, bufs) -> Optional[L.sbr_param_grads]:
    """sbr_param_grads for (materials, radar, rot, attenuation) gradient
    buffers (each None or contiguous float32 device memory of 2 n_mats, 6, 9
    and 1 elements), or None when all are None."""
    if bufs is None or all(t is None for t in bufs):
        return None
    for t, n in zip(bufs, (2 * len(mesh.materials or []), 6, 9, 1)):
        if t is not None:
            _buf(t, torch.float32, n, "parameter gradient")
            if t.numel() != n:
                raise ValueError(f"parameter gradient buffer must be contiguous float32 with {n} elements")
    return L.sbr_param_grads(*[t.data_ptr() if t is not None else None for t in bufs])


def sbr_backward(mesh: DeviceMesh, radar: S.Radar, rays: S.Grid, hits: Hits, chirp: S.Chirp, flags: int,
                 grad_if: torch.Tensor, grad_verts: torch.Tensor, scratch: torch.Tensor,
                 grad_materials: Optional[torch.Tensor] = None, grad_radar: Optional[torch.Tensor] = None,
                 grad_rot: Optional[torch.Tensor] = None, grad_atten: Optional[torch.Tensor] = None):
    m, r, g, h, c = mesh.struct(), radar_struct(radar), rays_struct(rays), hits.struct(), chirp_struct(chirp)
    mats, nm = materials_struct(mesh.materials)
    pg = _param_grads(mesh, (grad_materials, grad_radar, grad_rot, grad_atten))
    _check_hits(hits, rays.max_bounces, rays.nx * rays.ny)
    gi = _buf(grad_if, torch.float32, 2 * radar.n_virtual * chirp.n_chirps * chirp.n_samples, "grad_if")
    gv = _buf(grad_verts, torch.float32, 3 * mesh.nv, "grad_verts")
    L.check(_lib().sbr_backward(ct.byref(m), mats, nm, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c),
                                int(flags), gi, gv, ct.byref(pg) if pg is not None else None,
                                _buf(scratch, torch.uint8, 0, "scratch"), scratch.numel() * scratch.element_size(),
                                _stream()))


def sbr_loss_grad(mode: int, a: torch.Tensor, b: torch.Tensor, n: int, grad: Optional[torch.Tensor],
                  loss: Optional[torch.Tensor], scratch: Optional[torch.Tensor] = None):
    if loss is not None and scratch is None:
        scratch = torch.empty(L.SBR_LOSS_SCRATCH_BYTES, dtype=torch.uint8, device=a.device)
    nbytes = scratch.numel() * scratch.element_size() if scratch is not None else 0
    ap = _buf(a, torch.float32, 2 * n, "a")
    bp = _buf(b, torch.float32, (2 if mode == 0 else 1) * n, "b")
    L.check(_lib().sbr_loss_grad(int(mode), ap, bp, int(n), _buf(grad, torch.float32, 2 * n, "grad", optional=True),
                                 _buf(loss, torch.float32, 1, "loss", optional=True), _p(scratch), nbytes,
                                 _stream()))


def sbr_batch_table_bytes(n: int) -> int:
    return int(_lib().sbr_batch_table_bytes(int(n)))


def _request(mesh: DeviceMesh, radar: S.Radar, rays: S.Grid, hits: Hits, chirp: S.Chirp, flags: int,
             scratch: torch.Tensor, keep: list, if_cube: Optional[torch.Tensor] = None,
             grad_if: Optional[torch.Tensor] = None, grad_verts: Optional[torch.Tensor] = None,
             params=None) -> L.sbr_request:
    """One sbr_request after the buffer checks of the single-request calls;
    `keep` holds the ctypes structs it points to for the duration of the call."""
    V, C, Sn = radar.n_virtual, chirp.n_chirps, chirp.n_samples
    _check_hits(hits, rays.max_bounces, rays.nx * rays.ny)
    m, r, g, h, c = mesh.struct(), radar_struct(radar), rays_struct(rays), hits.struct(), chirp_struct(chirp)
    mats, nm = materials_struct(mesh.materials)
    keep.extend([m, r, g, h, c, mats])
    q = L.sbr_request()
    q.mesh, q.radar, q.rays, q.hits, q.chirp = ct.pointer(m), ct.pointer(r), ct.pointer(g), ct.pointer(h), ct.pointer(c)
    if mats is not None:
        q.mats = ct.cast(mats, ct.POINTER(L.sbr_material))
    q.n_mats, q.flags = nm, int(flags)
    q.if_cube = _buf(if_cube, torch.float32, 2 * V * C * Sn, "if_cube") if if_cube is not None else None
    q.grad_if = _buf(grad_if, torch.float32, 2 * V * C * Sn, "grad_if") if grad_if is not None else None
    q.grad_verts = _buf(grad_verts, torch.float32, 3 * mesh.nv, "grad_verts") if grad_verts is not None else None
    q.scratch = _buf(scratch, torch.uint8, 0, "scratch")
    q.scratch_bytes = scratch.numel() * scratch.element_size()
    pg = _param_grads(mesh, params)
    if pg is not None:
        keep.append(pg)
        q.params = ct.pointer(pg)
    return q


def sbr_synth_if_batched(items: Sequence[tuple], table: torch.Tensor):
    """items: (mesh, radar, rays, hits, chirp, flags, if_cube, scratch) per
    request; one batched synthesis on the current stream."""
    keep: list = []
    arr = (L.sbr_request * max(1, len(items)))()
    for i, (mesh, radar, rays, hits, chirp, flags, if_cube, scratch) in enumerate(items):
        arr[i] = _request(mesh, radar, rays, hits, chirp, flags, scratch, keep, if_cube=if_cube)
    L.check(_lib().sbr_synth_if_batched(arr, len(items), _buf(table, torch.uint8, 0, "table"),
                                        table.numel() * table.element_size(), _stream()))


def sbr_backward_batched(items: Sequence[tuple], table: torch.Tensor):
    """items: (mesh, radar, rays, hits, chirp, flags, grad_if, grad_verts,
    scratch[, params]) per request, params an optional (grad_materials,
    grad_radar, grad_rot, grad_atten) tuple as for sbr_backward; one batched
    backward pass on the current stream."""
    keep: list = []
    arr = (L.sbr_request * max(1, len(items)))()
    for i, it in enumerate(items):
        mesh, radar, rays, hits, chirp, flags, grad_if, grad_verts, scratch = it[:9]
        arr[i] = _request(mesh, radar, rays, hits, chirp, flags, scratch, keep, grad_if=grad_if,
                          grad_verts=grad_verts, params=it[9] if len(it) > 9 else None)
    L.check(_lib().sbr_backward_batched(arr, len(items), _buf(table, torch.uint8, 0, "table"),
                                        table.numel() * table.element_size(), _stream()))


def sbr_profile(op: int):
    L.check(_lib().sbr_profile(int(op)))


def sbr_profile_read(kernel: int):
    """(summed milliseconds, launches) of the recorded launches of one kernel."""
    ms, n = ct.c_double(), ct.c_int64()
    L.check(_lib().sbr_profile_read(int(kernel), ct.byref(ms), ct.byref(n)))
    return ms.value, n.value


def last_error() -> str:
    return _lib().sbr_last_error().decode()


# ----------------------------------------------------------------- convenience
def _angle_grid(rd: S.Radar, n_angle: int):
    """(n_ax, n_ay, n_angle) of the radar cube: a planar array's angle grid is
    n_ay x n_ax over the (TX, RX) = (vy, vx) virtual grid."""
    if getattr(rd, "planar", False):
        n_ax, n_ay = max(n_angle, rd.n_rx), max(n_angle, rd.n_tx)
        return n_ax, n_ay, n_ax * n_ay
    n = max(n_angle, rd.n_virtual)
    return n, 1, n


def _scratch_parts(scene: S.Scene, nf: Optional[int], backward: bool, cube: bool, n_angle: int):
    """(main, cube) bytes of a Simulator's two scratch buffers: the main one
    for the BVH build, the synthesis and (when asked for) the backward pass,
    which lay their path records out alike; the other for the radar cube and
    CFAR (when asked for), kept apart so that those stages do not overwrite
    the records between a synthesis and its backward pass."""
    g, rd, ch = scene.grid, scene.radar, scene.chirp
    nf = scene.nf if nf is None else nf
    m = L.sbr_mesh(None, scene.nv, None, nf, None)
    lib = _lib()
    rs, rr, cs = rays_struct(g), radar_struct(rd), chirp_struct(ch)
    main = max(int(lib.sbr_scratch_bytes(L.SBR_OP_BUILD_BVH, ct.byref(m), None, None, None)),
               int(lib.sbr_scratch_bytes(L.SBR_OP_SYNTH, ct.byref(m), ct.byref(rs), ct.byref(rr), ct.byref(cs))))
    if backward:
        main = max(main, int(lib.sbr_scratch_bytes(L.SBR_OP_BACKWARD, ct.byref(m), ct.byref(rs), ct.byref(rr),
                                                   ct.byref(cs))))
    cb = 0
    if cube:
        n_ax, n_ay, na = _angle_grid(rd, n_angle)
        C, Sn = ch.n_chirps, ch.n_samples
        cb = max(int(lib.sbr_scratch_bytes(L.SBR_OP_RADAR_CUBE, None, ct.byref(rs), ct.byref(rr), ct.byref(cs))),
                 int(lib.sbr_scratch_bytes(L.SBR_OP_CFAR, None, ct.byref(rs), ct.byref(rr), ct.byref(cs))))
        # the cube stage needs room for max(V, n_angle) planes
        if getattr(rd, "planar", False):
            cb = max(cb, sbr_radar_cube_2d_bytes(rd.n_rx, rd.n_tx, C, Sn, n_ax, n_ay))
        else:
            cb = max(cb, 2 * 8 * na * C * Sn + 1024)
    return main, cb


def simulator_scratch_bytes(scene: S.Scene, nf: Optional[int] = None, backward: bool = True, cube: bool = True,
                            n_angle: int = 64) -> int:
    """Bytes of the scratch a Simulator allocates: the largest of the stages
    it may run (BVH build and synthesis always, the backward pass when asked
    for) plus, when asked for, a separate buffer for the radar cube and CFAR."""
    main, cb = _scratch_parts(scene, nf, backward, cube, n_angle)
    return main + cb


class Simulator:
    """One scene resident on the device: mesh, BVH, hit records and scratch
    (stages on one stream run in order).  The main scratch serves the BVH
    build, the synthesis and, with `backward`, sbr_backward; with `cube` a
    second one serves the radar cube, CFAR and point clouds, so that the path
    records of a synthesis survive them and its backward pass can reuse them
    (`backward(..., reuse_paths=True)`)."""

    def __init__(self, scene: S.Scene, device="cuda", drop_flagged: bool = True, n_angle: int = 64,
                 mesh: Optional[DeviceMesh] = None, bvh: Optional[torch.Tensor] = None, exit_only: bool = False,
                 backward: bool = True, cube: bool = True):
        self.scene = scene
        self.device = torch.device(device)
        self.mesh = mesh if mesh is not None else DeviceMesh.from_scene(scene, self.device)
        self.flags = (L.SBR_DROP_FLAGGED if drop_flagged else 0) | (L.SBR_EXIT_ONLY if exit_only else 0)
        g, rd, ch = scene.grid, scene.radar, scene.chirp
        self.K, self.R = g.max_bounces, g.nx * g.ny
        self.V, self.C, self.S = rd.n_virtual, ch.n_chirps, ch.n_samples
        self.planar = bool(getattr(rd, "planar", False))
        self.n_ax, self.n_ay, self.n_angle = _angle_grid(rd, n_angle)
        main, cb = _scratch_parts(scene, self.mesh.nf, backward, cube, n_angle)
        self.scratch = torch.empty(main, dtype=torch.uint8, device=self.device)
        self.cube_scratch = torch.empty(cb, dtype=torch.uint8, device=self.device) if cube else None
        # identifies the synthesis whose path records the main scratch holds;
        # None once the mesh, BVH or hits may have changed since
        self.paths_token: Optional[int] = None
        self._n_synth = 0
        self.bvh = bvh if bvh is not None else torch.empty(max(1, sbr_bvh_bytes(self.mesh.nf)), dtype=torch.uint8,
                                                           device=self.device)
        self.hits = Hits.empty(self.K, self.R, self.device)
        self.counters = torch.zeros(3, dtype=torch.int64, device=self.device)
        self.loss_scratch = torch.empty(L.SBR_LOSS_SCRATCH_BYTES, dtype=torch.uint8, device=self.device)
        self.built = bvh is not None

    # ---- geometry
    def set_verts(self, verts: torch.Tensor):
        self.paths_token = None
        self.mesh.verts.copy_(verts.detach().to(torch.float32).reshape(-1, 3))

    def build(self, refit: bool = False):
        if self.mesh.nf == 0:
            return
        sbr_build_bvh(self.mesh, self.bvh, 1 if (refit and self.built) else 0, self.scratch)
        self.built = True
        self.paths_token = None

    # ---- forward
    def trace(self, count: bool = False):
        if not self.built:
            self.build()
        self.paths_token = None
        sbr_trace(self.mesh, self.bvh if self.mesh.nf else None, self.scene.radar, self.scene.grid, self.hits,
                  self.counters if count else None)
        return self.hits

    def synth(self, out: Optional[torch.Tensor] = None, direct_sums: bool = False) -> torch.Tensor:
        """IF cube (Eq. 8) of the current hits.  direct_sums=True sums over the
        paths directly instead of by the non-uniform FFT form."""
        if out is None:
            out = torch.empty((self.V, self.C, self.S, 2), dtype=torch.float32, device=self.device)
        flags = self.flags | (L.SBR_DIRECT_SUMS if direct_sums else 0)
        sbr_synth_if(self.mesh, self.scene.radar, self.scene.grid, self.hits, self.scene.chirp, flags, out,
                     self.scratch)
        self._n_synth += 1
        self.paths_token = self._n_synth
        return out

    def forward(self) -> torch.Tensor:
        self.trace()
        return torch.view_as_complex(self.synth())

    def _cube_scratch(self) -> torch.Tensor:
        if self.cube_scratch is None:
            raise RuntimeError("this Simulator was made with cube=False (no radar-cube scratch)")
        return self.cube_scratch

    def radar_cube(self, x: torch.Tensor, direction: int = 0, window: int = 0) -> torch.Tensor:
        xf = torch.view_as_real(x) if x.is_complex() else x
        xf = xf.contiguous()
        if direction == 0:
            out = torch.empty((self.n_angle, self.C, self.S, 2), dtype=torch.float32, device=self.device)
        else:
            out = torch.empty((self.V, self.C, self.S, 2), dtype=torch.float32, device=self.device)
        if self.planar:
            rd = self.scene.radar
            sbr_radar_cube_2d(xf, rd.n_rx, rd.n_tx, self.C, self.S, self.n_ax, self.n_ay, window, direction, out,
                              self._cube_scratch())
        else:
            sbr_radar_cube(xf, self.V, self.C, self.S, self.n_angle, window, direction, out, self._cube_scratch())
        return torch.view_as_complex(out)

    def cfar(self, X: torch.Tensor, guard=2, train=8, pfa=1e-4, max_points=65536):
        xf = (torch.view_as_real(X) if X.is_complex() else X).contiguous()
        pts = torch.empty((max_points, 4), dtype=torch.int32, device=self.device)
        ratio = torch.empty(max_points, dtype=torch.float32, device=self.device)
        n = torch.zeros(1, dtype=torch.int32, device=self.device)
        sbr_cfar(xf, int(xf.shape[0]), self.C, self.S, guard, train, pfa, pts, ratio, n, self._cube_scratch())
        return pts, ratio, n

    def cloud(self, points: torch.Tensor, n_points: torch.Tensor) -> torch.Tensor:
        """CFAR detections ([max_points, 4] int32 + device count) of this
        simulator's radar cube -> world points [max_points, 4] (x, y, z,
        radial velocity); rows past the count are NaN."""
        out = torch.empty((points.shape[0], 4), dtype=torch.float32, device=self.device)
        n_ax, n_ay = (self.n_ax, self.n_ay) if self.planar else (self.n_angle, 1)
        sbr_cloud(points, n_points, self.scene.radar, self.scene.chirp, n_ax, n_ay, out)
        return out

    def angle_peaks(self, X: torch.Tensor, det: torch.Tensor, n_det: torch.Tensor, rel: float = 0.1,
                    max_points: int = 65536):
        """Angle peaks (>= rel of each cell's strongest) of CFAR detections."""
        n_ax, n_ay = (self.n_ax, self.n_ay) if self.planar else (self.n_angle, 1)
        return sbr_angle_peaks(X, n_ax, n_ay, self.C, self.S, det, n_det, rel, max_points)

    def point_cloud(self, cube: torch.Tensor, guard: int = 2, train: int = 8, pfa: float = 1e-4,
                    max_points: int = 65536, window: int = 1, rel: Optional[float] = 0.1,
                    snr_db: Optional[float] = 20.0, seed: int = 0) -> torch.Tensor:
        """IF cube -> radar cube (Hann window) -> CA-CFAR over range-Doppler ->
        angle peaks (rel=None: only each cell's strongest angle) -> world
        points [n, 4] (x, y, z, radial velocity): the point cloud a radar
        reports.  snr_db adds seeded complex receiver noise at that ratio to
        the cube's RMS sample power first (None: none); without a noise floor
        the CFAR of a noise-free synthetic cube fires on DFT sidelobes."""
        if snr_db is not None:
            g = torch.Generator(device=self.device).manual_seed(seed)
            shape = cube.shape if cube.is_complex() else cube.shape[:-1]
            cc = cube if cube.is_complex() else torch.view_as_complex(cube.contiguous())
            rms = cc.abs().pow(2).mean().sqrt()
            noise = torch.complex(torch.randn(shape, generator=g, device=self.device),
                                  torch.randn(shape, generator=g, device=self.device)) * (0.7071067811865476 *
                                                                                           10 ** (-snr_db / 20))
            cube = cc + noise.to(cc.dtype) * rms
        X = self.radar_cube(cube, window=window)
        det, _, nd = self.cfar(X, guard, train, pfa, 4096)
        if rel is not None:
            det, nd = self.angle_peaks(X, det, nd, rel, max_points)
        xyz = self.cloud(det, nd)
        return xyz[: min(int(nd.item()), det.shape[0])]

    def backward(self, grad_if: torch.Tensor, grad_verts: Optional[torch.Tensor] = None,
                 grad_materials: Optional[torch.Tensor] = None, grad_radar: Optional[torch.Tensor] = None,
                 grad_rot: Optional[torch.Tensor] = None, attached: bool = False,
                 grad_atten: Optional[torch.Tensor] = None, direct_sums: bool = False,
                 reuse_paths: bool = False) -> torch.Tensor:
        """dL/dverts (accumulated into grad_verts); optionally also accumulates
        dL/d(eps_r, sigma) per material [n_mats,2], dL/d(origin, velocity) [6]
        dL/d rot [3,3] (radar -> world, row-major) and dL/d attenuation [1].  attached=True
        differentiates the reparameterised estimator (samples follow their
        first hit, Eqs. 6-7), so that moving silhouettes contribute.
        direct_sums=True sums the per-path adjoint series of Eqs. 11-12
        directly over the samples instead of by the non-uniform FFT.
        reuse_paths=True takes the path records of the last synth() from the
        scratch instead of recomputing them (SBR_PATHS_IN_SCRATCH); it is an
        error once build(), trace() or set_verts() has run since.  The scene's
        radar and chirp must be the ones that synthesis used."""
        gf = (torch.view_as_real(grad_if) if grad_if.is_complex() else grad_if).contiguous().to(torch.float32)
        if grad_verts is None:
            grad_verts = torch.zeros((self.mesh.nv, 3), dtype=torch.float32, device=self.device)
        flags = self.flags | (L.SBR_ATTACHED if attached else 0) | (L.SBR_DIRECT_SUMS if direct_sums else 0)
        if reuse_paths:
            if self.paths_token is None:
                raise RuntimeError("reuse_paths: the scratch holds no path records of the current hits")
            flags |= L.SBR_PATHS_IN_SCRATCH
        sbr_backward(self.mesh, self.scene.radar, self.scene.grid, self.hits, self.scene.chirp, flags, gf,
                     grad_verts, self.scratch, grad_materials, grad_radar, grad_rot, grad_atten)
        return grad_verts

    def loss_grad(self, cube: torch.Tensor, target: torch.Tensor, grad: Optional[torch.Tensor] = None,
                  loss: Optional[torch.Tensor] = None, mode: int = 0):
        """IF loss sum |S - target|^2 (mode 0) or heatmap MSE (mode 1) and its gradient."""
        a = (torch.view_as_real(cube) if cube.is_complex() else cube).contiguous()
        b = (torch.view_as_real(target) if target.is_complex() else target).contiguous()
        n = a.numel() // 2
        if grad is None:
            grad = torch.empty_like(a)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        sbr_loss_grad(mode, a, b, n, grad, loss, self.loss_scratch)
        return grad, loss

    def n_paths(self) -> int:
        return int(self.scratch[:4].view(torch.int32)[0].item())
