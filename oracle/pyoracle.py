"""ctypes front end of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use this module.  It loads `oracle/liboracle.so` (plain C99, built
from `oracle/oracle.c` with gcc) and shares nothing with the HIP library.

Gradients are checked against central finite differences of the oracle's
loss with the hit-triangle sequence of every ray frozen (the pathwise
derivative of the fixed-grid estimator, paper Sec. 3.2.1, Eqs. (4)-(5) and
Sec. 3.3, Eq. (13)); rays whose hits lie within 1e-6 m of an edge are
flagged by the trace and dropped, which is where a frozen sequence could
differ from a re-trace.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

F_EDGE, F_TIE, F_GRAZE, F_TMIN, F_PARENT, F_OCCLUDED = 1, 2, 4, 8, 16, 32
DROP_FLAGGED, EXIT_ONLY = 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Mesh(ct.Structure):
    _fields_ = [("nv", ct.c_int), ("nf", ct.c_int), ("verts", ct.POINTER(ct.c_double)),
                ("faces", ct.POINTER(ct.c_int)), ("mat_id", ct.POINTER(ct.c_int)),
                ("n_mats", ct.c_int), ("mat_mode", ct.POINTER(ct.c_int)),
                ("mat_eps_r", ct.POINTER(ct.c_double)), ("mat_sigma", ct.POINTER(ct.c_double))]


class _Radar(ct.Structure):
    _fields_ = [("origin", ct.c_double * 3), ("rot", ct.c_double * 9), ("n_tx", ct.c_int),
                ("n_rx", ct.c_int), ("tx", (ct.c_double * 3) * 20), ("rx", (ct.c_double * 3) * 20),
                ("vel", ct.c_double * 3), ("atten", ct.c_double), ("n_tx_gain", ct.c_double),
                ("n_rx_gain", ct.c_double)]


class _Chirp(ct.Structure):
    _fields_ = [("fc", ct.c_double), ("slope", ct.c_double), ("fs", ct.c_double),
                ("t_chirp", ct.c_double), ("n_samples", ct.c_int), ("n_chirps", ct.c_int)]


class _Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("tan_hx", ct.c_double),
                ("tan_hy", ct.c_double), ("max_bounces", ct.c_int), ("t_min", ct.c_double),
                ("shadow", ct.c_int), ("jitter", ct.c_int), ("seed_lo", ct.c_uint), ("seed_hi", ct.c_uint)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ct.CDLL(LIB_PATH)
        dp, ip, bp = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int), ct.POINTER(ct.c_ubyte)
        L.orc_philox4x32_10.argtypes = [ct.POINTER(ct.c_uint), ct.POINTER(ct.c_uint), ct.POINTER(ct.c_uint)]
        L.orc_ray.argtypes = [ct.POINTER(_Radar), ct.POINTER(_Grid), ct.c_int, dp, dp, dp]
        L.orc_trace.restype = ct.c_longlong
        L.orc_trace.argtypes = [ct.POINTER(_Mesh), ct.POINTER(_Radar), ct.POINTER(_Grid), ip,
                                ct.c_int, ip, dp, dp, dp, bp, bp, dp]
        L.orc_fresnel.argtypes = [ct.POINTER(_Mesh), ct.c_int, ct.c_double, ct.c_double, dp]
        L.orc_paths.restype = ct.c_int
        L.orc_paths.argtypes = [ct.POINTER(_Mesh), ct.POINTER(_Radar), ct.POINTER(_Grid),
                                ct.POINTER(_Chirp), ip, ct.c_int, ip, bp, ct.c_int, dp, ip, ip, dp, dp,
                                dp, dp]
        L.orc_attach.argtypes = [ct.POINTER(_Mesh), ct.POINTER(_Radar), ct.POINTER(_Grid), ip, ct.c_int,
                                 ip, dp]
        L.orc_synth.argtypes = [ct.c_int, dp, dp, dp, ct.c_int, ct.POINTER(_Chirp), ip, ct.c_int, dp]
        L.orc_synth_adjoint.argtypes = [ct.c_int, dp, dp, dp, ct.c_int, ct.POINTER(_Chirp), dp,
                                        dp, dp, dp]
        L.orc_radar_cube.argtypes = [dp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                     ct.c_int, dp]
        L.orc_radar_cube2.argtypes = [dp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                      ct.c_int, ct.c_int, dp]
        L.orc_angle_peaks.restype = ct.c_int
        L.orc_angle_peaks.argtypes = [dp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ip, ct.c_int, ct.c_double, ip,
                                      ct.c_int]
        L.orc_cloud.argtypes = [ip, ct.c_int, ct.POINTER(_Radar), ct.POINTER(_Chirp), ct.c_int, ct.c_int, dp]
        L.orc_cfar.restype = ct.c_int
        L.orc_cfar.argtypes = [dp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_double,
                               bp, ip, dp, dp]
        _lib = L
    return _lib


def _p(a, typ):
    return a.ctypes.data_as(ct.POINTER(typ)) if a is not None else None


class _Keep:
    """Holds numpy buffers alive while a struct points into them."""

    def __init__(self):
        self.bufs = []

    def add(self, a):
        self.bufs.append(a)
        return a


def _mesh(scene, verts64=None, keep=None):
    keep = keep if keep is not None else _Keep()
    v = keep.add(np.ascontiguousarray(scene.verts.astype(np.float64) if verts64 is None else verts64,
                                      dtype=np.float64))
    f = keep.add(np.ascontiguousarray(scene.faces, dtype=np.int32))
    m = _Mesh()
    m.nv, m.nf = v.shape[0], f.shape[0]
    m.verts, m.faces = _p(v, ct.c_double), _p(f, ct.c_int)
    if scene.materials:
        mid = keep.add(np.ascontiguousarray(
            scene.mat_id if scene.mat_id is not None else np.zeros(m.nf), dtype=np.int32))
        mode = keep.add(np.array([x[0] for x in scene.materials], np.int32))
        er = keep.add(np.array([x[1] for x in scene.materials], np.float64))
        sg = keep.add(np.array([x[2] for x in scene.materials], np.float64))
        m.mat_id, m.n_mats = _p(mid, ct.c_int), len(scene.materials)
        m.mat_mode, m.mat_eps_r, m.mat_sigma = _p(mode, ct.c_int), _p(er, ct.c_double), _p(sg, ct.c_double)
    else:
        m.mat_id, m.n_mats = None, 0
    return m, keep


def _radar(rd):
    r = _Radar()
    for i in range(3):
        r.origin[i] = float(rd.origin[i])
        r.vel[i] = float(rd.vel[i])
    for i in range(9):
        r.rot[i] = float(np.asarray(rd.rot).reshape(-1)[i])
    r.n_tx, r.n_rx = rd.n_tx, rd.n_rx
    r.atten = float(getattr(rd, "atten", 0.0))
    r.n_tx_gain = float(getattr(rd, "n_tx_gain", 0.0))
    r.n_rx_gain = float(getattr(rd, "n_rx_gain", 0.0))
    for t in range(rd.n_tx):
        for j in range(3):
            r.tx[t][j] = float(rd.tx[t][j])
    for q in range(rd.n_rx):
        for j in range(3):
            r.rx[q][j] = float(rd.rx[q][j])
    return r


def _chirp(ch):
    return _Chirp(ch.fc, ch.slope, ch.fs, ch.t_chirp, ch.n_samples, ch.n_chirps)


def _grid(g):
    seed = getattr(g, "jitter_seed", None)
    return _Grid(g.nx, g.ny, g.tan_hx, g.tan_hy, g.max_bounces, g.t_min, int(getattr(g, "shadow", False)),
                 int(seed is not None), (seed or 0) & 0xFFFFFFFF, ((seed or 0) >> 32) & 0xFFFFFFFF)


def philox4x32_10(ctr, key):
    c = (ct.c_uint * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ct.c_uint * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ct.c_uint * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def ray(scene, r):
    o, d, w = (ct.c_double * 3)(), (ct.c_double * 3)(), ct.c_double()
    lib().orc_ray(ct.byref(_radar(scene.radar)), ct.byref(_grid(scene.grid)), int(r), o, d, ct.byref(w))
    return np.array(o[:]), np.array(d[:]), w.value


def trace(scene, rays=None, verts64=None):
    """Brute-force closest hits.  Returns dict of [K][n] arrays + query count."""
    g = scene.grid
    K = g.max_bounces
    ids = None if rays is None else np.ascontiguousarray(rays, dtype=np.int32)
    n = g.n_rays if ids is None else len(ids)
    tri = np.empty((K, n), np.int32)
    t = np.empty((K, n))
    b1 = np.empty((K, n))
    b2 = np.empty((K, n))
    fl = np.empty((K, n), np.uint8)
    se = np.empty((K, n), np.uint8)
    cs = np.empty((K, n))
    m, keep = _mesh(scene, verts64)
    q = lib().orc_trace(ct.byref(m), ct.byref(_radar(scene.radar)), ct.byref(_grid(g)),
                        _p(ids, ct.c_int), n, _p(tri, ct.c_int), _p(t, ct.c_double),
                        _p(b1, ct.c_double), _p(b2, ct.c_double), _p(fl, ct.c_ubyte), _p(se, ct.c_ubyte),
                        _p(cs, ct.c_double))
    return {"tri": tri, "t": t, "b1": b1, "b2": b2, "flags": fl, "shadow_edge": se, "cos": cs, "queries": int(q)}


def attach(scene, tri, rays=None, verts64=None):
    """(b1, b2, D0) per ray of the first hit (Eqs. 6-7 transform attached to
    it); tri is the [K][n] hit-id array of the unperturbed scene."""
    ids = None if rays is None else np.ascontiguousarray(rays, dtype=np.int32)
    t0 = np.ascontiguousarray(tri[0], dtype=np.int32)
    out = np.empty((len(t0), 3))
    m, keep = _mesh(scene, verts64)
    lib().orc_attach(ct.byref(m), ct.byref(_radar(scene.radar)), ct.byref(_grid(scene.grid)),
                     _p(ids, ct.c_int), len(t0), _p(t0, ct.c_int), _p(out, ct.c_double))
    return out


def paths(scene, tri, flags=None, rays=None, drop=True, verts64=None, att=None, exit_only=False):
    """Per-path amplitude, delays and Doppler from frozen hit ids.  att: None
    (fixed ray directions) or the per-ray array of attach() (first hit at
    fixed barycentrics, cell weight times |det J_T|).  Occluded records never
    return; drop skips the other flagged ones; exit_only keeps only the last
    hit of each ray."""
    g = scene.grid
    K = g.max_bounces
    V = scene.radar.n_virtual
    ids = None if rays is None else np.ascontiguousarray(rays, dtype=np.int32)
    n = tri.shape[1]
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    cap = max(1, K * n)
    pr = np.empty(cap, np.int32)
    pk = np.empty(cap, np.int32)
    amp = np.empty((cap, 2))
    tau = np.empty((cap, V))
    td = np.empty(cap)
    wt = np.empty(cap)
    at = None if att is None else np.ascontiguousarray(att, dtype=np.float64)
    m, keep = _mesh(scene, verts64)
    P = lib().orc_paths(ct.byref(m), ct.byref(_radar(scene.radar)), ct.byref(_grid(g)),
                        ct.byref(_chirp(scene.chirp)), _p(ids, ct.c_int), n, _p(tri, ct.c_int),
                        _p(fl, ct.c_ubyte), (DROP_FLAGGED if drop and fl is not None else 0) |
                        (EXIT_ONLY if exit_only else 0), _p(at, ct.c_double),
                        _p(pr, ct.c_int), _p(pk, ct.c_int), _p(amp, ct.c_double), _p(tau, ct.c_double),
                        _p(td, ct.c_double), _p(wt, ct.c_double))
    return {"ray": pr[:P].copy(), "k": pk[:P].copy(), "amp": amp[:P, 0] + 1j * amp[:P, 1],
            "tau": tau[:P].copy(), "taudot": td[:P].copy(), "weight": wt[:P].copy()}


def synth(scene, pth, rows=None):
    """Eq. (8) IF cube [V][C][S] (complex128), or [len(rows)][S] for a row subset."""
    ch = scene.chirp
    V = scene.radar.n_virtual
    C, S = ch.n_chirps, ch.n_samples
    P = len(pth["amp"])
    amp = np.ascontiguousarray(np.stack([pth["amp"].real, pth["amp"].imag], -1)).reshape(-1) if P else np.zeros(2)
    tau = np.ascontiguousarray(pth["tau"], dtype=np.float64).reshape(-1) if P else np.zeros(V)
    td = np.ascontiguousarray(pth["taudot"], dtype=np.float64) if P else np.zeros(1)
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    nr = V * C if rws is None else len(rws)
    out = np.empty((nr, S, 2))
    lib().orc_synth(P, _p(amp, ct.c_double), _p(tau, ct.c_double), _p(td, ct.c_double), V,
                    ct.byref(_chirp(ch)), _p(rws, ct.c_int), nr, _p(out, ct.c_double))
    cube = out[..., 0] + 1j * out[..., 1]
    return cube.reshape(V, C, S) if rws is None else cube


def synth_adjoint(scene, pth, G):
    ch = scene.chirp
    V = scene.radar.n_virtual
    P = len(pth["amp"])
    amp = np.ascontiguousarray(np.stack([pth["amp"].real, pth["amp"].imag], -1)).reshape(-1)
    tau = np.ascontiguousarray(pth["tau"], dtype=np.float64)
    td = np.ascontiguousarray(pth["taudot"], dtype=np.float64)
    g = np.ascontiguousarray(np.stack([G.real, G.imag], -1), dtype=np.float64)
    ab = np.empty((P, 2))
    tb = np.empty((P, V))
    tdb = np.empty(P)
    lib().orc_synth_adjoint(P, _p(amp, ct.c_double), _p(tau, ct.c_double), _p(td, ct.c_double), V,
                            ct.byref(_chirp(ch)), _p(g, ct.c_double), _p(ab, ct.c_double),
                            _p(tb, ct.c_double), _p(tdb, ct.c_double))
    return ab[:, 0] + 1j * ab[:, 1], tb, tdb


def radar_cube(x, n_angle=64, window=0, direction=0, V=None):
    """direction 0: [V][C][S] -> [Na][C][S];  1: [Na][C][S] -> [V][C][S]."""
    x = np.asarray(x, np.complex128)
    if direction == 0:
        V_, C, S = x.shape
        out = np.empty((n_angle, C, S, 2))
    else:
        _, C, S = x.shape
        V_ = V
        out = np.empty((V_, C, S, 2))
    inp = np.ascontiguousarray(np.stack([x.real, x.imag], -1))
    lib().orc_radar_cube(_p(inp, ct.c_double), V_, C, S, n_angle, window, direction,
                         _p(out, ct.c_double))
    return out[..., 0] + 1j * out[..., 1]


def radar_cube2(x, vx, vy, n_ax=64, n_ay=64, window=0, direction=0):
    """Planar array.  direction 0: [Vy*Vx][C][S] -> [Nay*Nax][C][S];  1: back."""
    x = np.asarray(x, np.complex128)
    _, C, S = x.shape
    n_out = n_ax * n_ay if direction == 0 else vx * vy
    out = np.empty((n_out, C, S, 2))
    inp = np.ascontiguousarray(np.stack([x.real, x.imag], -1))
    lib().orc_radar_cube2(_p(inp, ct.c_double), vx, vy, C, S, n_ax, n_ay, window, direction,
                          _p(out, ct.c_double))
    return out[..., 0] + 1j * out[..., 1]


def cfar(X, guard=2, train=8, pfa=1e-4):
    X = np.asarray(X, np.complex128)
    Na, C, S = X.shape
    inp = np.ascontiguousarray(np.stack([X.real, X.imag], -1))
    st = np.empty((C, S), np.uint8)
    am = np.empty((C, S), np.int32)
    pw = np.empty((C, S))
    rt = np.empty((C, S))
    n = lib().orc_cfar(_p(inp, ct.c_double), Na, C, S, guard, train, pfa, _p(st, ct.c_ubyte),
                       _p(am, ct.c_int), _p(pw, ct.c_double), _p(rt, ct.c_double))
    return {"count": n, "status": st, "argmax": am, "power": pw, "ratio": rt}


def angle_peaks(X, n_ax, n_ay, det, rel, max_out=1 << 20):
    """Angle peaks of the detected cells of cube X [Nay*Nax][C][S]."""
    X = np.asarray(X, np.complex128)
    _, C, S = X.shape
    inp = np.ascontiguousarray(np.stack([X.real, X.imag], -1))
    d = np.ascontiguousarray(det, dtype=np.int32).reshape(-1, 4)
    out = np.empty((max_out, 4), np.int32)
    n = lib().orc_angle_peaks(_p(inp, ct.c_double), n_ax, n_ay, C, S, _p(d, ct.c_int), len(d), float(rel),
                              _p(out, ct.c_int), max_out)
    return out[:min(n, max_out)].copy()


def cloud(scene, points, n_ax, n_ay=1):
    """[n][4] detections (range bin, Doppler bin, angle index, 0) -> [n][4]
    world x, y, z, radial velocity."""
    pts = np.ascontiguousarray(points, dtype=np.int32).reshape(-1, 4)
    out = np.empty((len(pts), 4))
    lib().orc_cloud(_p(pts, ct.c_int), len(pts), ct.byref(_radar(scene.radar)), ct.byref(_chirp(scene.chirp)),
                    n_ax, n_ay, _p(out, ct.c_double))
    return out


def fresnel(mode, eps_r, sigma, fc, cos_i):
    import types
    sc = types.SimpleNamespace(verts=np.zeros((1, 3)), faces=np.zeros((1, 3), np.int32),
                               materials=[(mode, eps_r, sigma)], mat_id=None)
    m, keep = _mesh(sc)
    out = (ct.c_double * 2)()
    lib().orc_fresnel(ct.byref(m), 0, fc, cos_i, out)
    return complex(out[0], out[1])


def forward(scene, rays=None, drop=True, exit_only=False):
    tr = trace(scene, rays)
    pth = paths(scene, tr["tri"], tr["flags"], rays, drop, exit_only=exit_only)
    return synth(scene, pth), tr, pth


def if_loss(S, target):
    d = S - target
    return float(np.sum(d.real ** 2 + d.imag ** 2))


def fd_directional(scene, tri, flags, target, direction, h=1e-9, rays=None, drop=True, att=None,
                   exit_only=False):
    """Central difference of L = sum |S - target|^2 along `direction` ([nv][3])
    with the hit-triangle sequences frozen (att: see paths())."""
    v0 = scene.verts.astype(np.float64)
    Ls = []
    for sgn in (+1.0, -1.0):
        p = paths(scene, tri, flags, rays, drop, verts64=v0 + sgn * h * direction, att=att, exit_only=exit_only)
        Ls.append(if_loss(synth(scene, p), target))
    return (Ls[0] - Ls[1]) / (2.0 * h)


def fd_scene(scene, tri, flags, target, perturb, h, rays=None, drop=True, att=None):
    """Central difference of the IF loss with respect to a scalar scene
    parameter: perturb(scene, delta) returns the scene with the parameter
    moved by delta (hit-triangle sequences frozen)."""
    Ls = []
    for sgn in (+1.0, -1.0):
        sp = perturb(scene, sgn * h)
        Ls.append(if_loss(synth(sp, paths(sp, tri, flags, rays, drop, att=att)), target))
    return (Ls[0] - Ls[1]) / (2.0 * h)


def fd_grad(scene, tri, flags, target, coords=None, h=1e-9, rays=None, drop=True, att=None, exit_only=False):
    """Central differences of the IF loss for every vertex coordinate in
    `coords` (flat indices into [nv*3]; None = all)."""
    nv = scene.nv
    coords = np.arange(nv * 3) if coords is None else np.asarray(coords)
    g = np.zeros(len(coords))
    for i, c in enumerate(coords):
        e = np.zeros((nv, 3))
        e.reshape(-1)[c] = 1.0
        g[i] = fd_directional(scene, tri, flags, target, e, h, rays, drop, att, exit_only)
    return g


def fd_retraced(scene, target, direction, h, rays=None):
    """Central difference of the IF loss along `direction` with the scene
    traced again at each side (hit sets free to change, nothing dropped): the
    derivative of the estimator itself, visibility changes included."""
    v0 = scene.verts.astype(np.float64)
    Ls = []
    for sgn in (+1.0, -1.0):
        v = v0 + sgn * h * direction
        tr = trace(scene, rays, verts64=v)
        p = paths(scene, tr["tri"], tr["flags"], rays, False, verts64=v)
        Ls.append(if_loss(synth(scene, p), target))
    return (Ls[0] - Ls[1]) / (2.0 * h)
