"""Seeded synthetic scenes: meshes, radar poses, antenna layouts, chirps, ray grids.

This module only generates *inputs*.  It holds none of the simulator's
arithmetic (no ray tracing, no path model, no signal synthesis), so both the
HIP path and the FP64 oracle may read what it produces.

Every scene is plain data shaped like the workloads of the paper's Sec. 5
(FMCW radars at 24-81 GHz with MIMO arrays, Sec. 4; single objects and
cluttered multi-object scenes), built from textbook procedural generators:
icosphere / geodesic subdivision of the icosahedron, superquadrics, and
Perlin gradient noise (Perlin, SIGGRAPH 2002, "Improving Noise").
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

C0 = 299792458.0

# material modes of the per-face material table
MAT_PEC, MAT_TE, MAT_TM = 0, 1, 2


@dataclasses.dataclass
class Chirp:
    fc: float = 77e9          # carrier, Hz
    slope: float = 60e12      # mu = B / T, Hz/s (60 MHz/us)
    fs: float = 10e6          # ADC rate, Hz
    t_chirp: float = 40e-6    # chirp repetition period, s
    n_samples: int = 256
    n_chirps: int = 1


@dataclasses.dataclass
class Grid:
    nx: int = 64
    ny: int = 64
    tan_hx: float = math.tan(math.radians(15.0))
    tan_hy: float = math.tan(math.radians(15.0))
    max_bounces: int = 3
    t_min: float = 1e-5
    shadow: bool = False          # occlusion test of every return after the first bounce
    jitter_seed: Optional[int] = None   # stratified Monte Carlo sample per cell (Eq. 4), 64-bit Philox key

    @property
    def n_rays(self) -> int:
        return self.nx * self.ny


@dataclasses.dataclass
class Radar:
    origin: np.ndarray                       # (3,) world
    rot: np.ndarray                          # (3,3) radar -> world, columns = x, y, z axes
    tx: np.ndarray                           # (n_tx, 3) radar frame
    rx: np.ndarray                           # (n_rx, 3) radar frame
    vel: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))  # scene velocity, world
    planar: bool = False                     # virtual antennas form an n_tx x n_rx grid (vy = t, vx = m)
    atten: float = 0.0                       # amplitude attenuation of the medium, 1/m (Eq. 5's A)
    n_tx_gain: float = 0.0                   # TX gain F = cos^n(angle to boresight), 0 = isotropic (Eq. 1)
    n_rx_gain: float = 0.0                   # RX gain G = cos^n(angle to boresight) of the return

    @property
    def n_tx(self) -> int:
        return int(self.tx.shape[0])

    @property
    def n_rx(self) -> int:
        return int(self.rx.shape[0])

    @property
    def n_virtual(self) -> int:
        return self.n_tx * self.n_rx


@dataclasses.dataclass
class Scene:
    name: str
    verts: np.ndarray                        # float32 (nv, 3)
    faces: np.ndarray                        # int32 (nf, 3)
    radar: Radar
    chirp: Chirp
    grid: Grid
    mat_id: Optional[np.ndarray] = None      # uint16 (nf,) or None (all conductor)
    materials: List[Tuple[int, float, float]] = dataclasses.field(default_factory=list)

    @property
    def nv(self) -> int:
        return int(self.verts.shape[0])

    @property
    def nf(self) -> int:
        return int(self.faces.shape[0])

    def with_verts(self, verts: np.ndarray) -> "Scene":
        return dataclasses.replace(self, verts=np.ascontiguousarray(verts, dtype=np.float32))

    def with_grid(self, **kw) -> "Scene":
        return dataclasses.replace(self, grid=dataclasses.replace(self.grid, **kw))

    def with_chirp(self, **kw) -> "Scene":
        return dataclasses.replace(self, chirp=dataclasses.replace(self.chirp, **kw))


# --------------------------------------------------------------------------- arrays
def wavelength(fc: float) -> float:
    return C0 / fc


def ula_array(n_tx: int, n_rx: int, fc: float) -> Tuple[np.ndarray, np.ndarray]:
    """TX spaced 2*lambda, RX spaced lambda/2 along the radar x axis: the
    virtual array is an n_tx*n_rx element lambda/2 ULA centred at the origin
    (the 3TX/4RX layout of the 77 GHz automotive class of Sec. 4)."""
    lam = wavelength(fc)
    tx = np.zeros((n_tx, 3))
    rx = np.zeros((n_rx, 3))
    tx[:, 0] = (np.arange(n_tx) - (n_tx - 1) / 2.0) * (n_rx * lam / 2.0)
    rx[:, 0] = (np.arange(n_rx) - (n_rx - 1) / 2.0) * (lam / 2.0)
    return tx, rx


def default_radar(n_tx: int = 1, n_rx: int = 4, fc: float = 77e9,
                  vel=(0.0, 0.0, 0.0)) -> Radar:
    tx, rx = ula_array(n_tx, n_rx, fc)
    return Radar(origin=np.zeros(3), rot=np.eye(3), tx=tx, rx=rx, vel=np.asarray(vel, float))


def planar_array(n_tx: int, n_rx: int, fc: float) -> Tuple[np.ndarray, np.ndarray]:
    """TX along the radar y axis and RX along x, both lambda/2 apart: the
    virtual array is an n_tx x n_rx lambda/2 grid centred at the origin (the
    20 TX x 20 RX imaging class of Sec. 4)."""
    lam = wavelength(fc)
    tx = np.zeros((n_tx, 3))
    rx = np.zeros((n_rx, 3))
    tx[:, 1] = (np.arange(n_tx) - (n_tx - 1) / 2.0) * (lam / 2.0)
    rx[:, 0] = (np.arange(n_rx) - (n_rx - 1) / 2.0) * (lam / 2.0)
    return tx, rx


def planar_radar(n_tx: int = 20, n_rx: int = 20, fc: float = 62e9, vel=(0.0, 0.0, 0.0)) -> Radar:
    tx, rx = planar_array(n_tx, n_rx, fc)
    return Radar(origin=np.zeros(3), rot=np.eye(3), tx=tx, rx=rx, vel=np.asarray(vel, float), planar=True)


def platform(name: str) -> Tuple[Radar, Chirp]:
    """Radar and chirp of the three FMCW platform classes of Sec. 4.  The paper
    gives each one's band and antenna counts only; the chirps here are
    choices that fit those bands (256 samples at 10 MHz in every case):
      "ranging_24g"    1 TX, 2 RX at 24 GHz, 200 MHz swept over the ADC window
      "automotive_77g" 3 TX, 4 RX lambda/2 ULA at 77 GHz, 60 MHz/us
      "imaging_62g"    20 TX x 20 RX planar grid at 62 GHz, 7 GHz swept"""
    window = 256 / 10e6
    if name == "ranging_24g":
        return default_radar(1, 2, 24.0e9), Chirp(fc=24.0e9, slope=200e6 / window)
    if name == "automotive_77g":
        return default_radar(3, 4, 77e9), Chirp(fc=77e9, slope=60e12)
    if name == "imaging_62g":
        return planar_radar(20, 20, 62e9), Chirp(fc=62e9, slope=7e9 / window, t_chirp=40e-6)
    raise ValueError(f"unknown platform {name!r}")


def fov_tan(radius: float, distance: float, margin: float = 1.02) -> float:
    """Half-width of the tangent grid that covers a bounding sphere."""
    return math.tan(math.asin(min(radius / distance, 0.999))) * margin


# --------------------------------------------------------------------------- meshes
def _dedupe(points: np.ndarray, faces: np.ndarray, decimals: int = 9):
    key = np.round(points, decimals)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    # keep the first original coordinates of each unique key
    first = np.full(len(uniq), -1, dtype=np.int64)
    for i in range(len(inv) - 1, -1, -1):
        first[inv[i]] = i
    return points[first], inv[faces]


def icosahedron() -> Tuple[np.ndarray, np.ndarray]:
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v, f


def icosphere(level: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit icosphere by `level` rounds of 1->4 midpoint subdivision."""
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    faces = f.tolist()
    for _ in range(level):
        cache = {}
        vl = verts

        def mid(a, b):
            k = (a, b) if a < b else (b, a)
            if k not in cache:
                p = (np.asarray(vl[a]) + np.asarray(vl[b])) / 2.0
                p /= np.linalg.norm(p)
                cache[k] = len(vl)
                vl.append(tuple(p))
            return cache[k]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        faces = nf
    return np.asarray(verts, np.float64), np.asarray(faces, np.int64)


def geodesic_sphere(freq: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit geodesic sphere: each icosahedron face split into freq^2 triangles
    on a barycentric lattice, vertices projected to the sphere
    (10 freq^2 + 2 vertices, 20 freq^2 faces)."""
    v, f = icosahedron()
    pts, tris = [], []
    base = 0
    for a, b, c in f:
        A, B, C = v[a], v[b], v[c]
        idx = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                p = A + (B - A) * (i / freq) + (C - A) * (j / freq)
                idx[(i, j)] = base + len(idx)
                pts.append(p / np.linalg.norm(p))
        for i in range(freq):
            for j in range(freq - i):
                tris.append([idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]])
                if i + j < freq - 1:
                    tris.append([idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]])
        base += len(idx)
    pts = np.asarray(pts)
    tris = np.asarray(tris, np.int64)
    return _dedupe(pts, tris)


def _sgnpow(x, e):
    return np.sign(x) * np.abs(x) ** e


def superquadric(n_lon: int, n_lat: int, axes, e1: float, e2: float):
    """Closed superquadric surface on a longitude/latitude grid with pole
    vertices: n_lon * (n_lat - 1) + 2 vertices, 2 n_lon (n_lat - 1) faces."""
    a1, a2, a3 = axes
    eta = -math.pi / 2 + math.pi * np.arange(1, n_lat) / n_lat        # rings
    om = -math.pi + 2 * math.pi * np.arange(n_lon) / n_lon
    E, W = np.meshgrid(eta, om, indexing="ij")
    x = a1 * _sgnpow(np.cos(E), e1) * _sgnpow(np.cos(W), e2)
    y = a2 * _sgnpow(np.cos(E), e1) * _sgnpow(np.sin(W), e2)
    z = a3 * _sgnpow(np.sin(E), e1)
    ring = np.stack([x, y, z], -1).reshape(-1, 3)
    south = np.array([[0.0, 0.0, -a3]])
    north = np.array([[0.0, 0.0, a3]])
    verts = np.concatenate([ring, south, north])
    S, N = len(ring), len(ring) + 1
    nr = n_lat - 1
    i, j = np.meshgrid(np.arange(nr - 1), np.arange(n_lon), indexing="ij")
    j2 = (j + 1) % n_lon
    a, b = i * n_lon + j, i * n_lon + j2
    c, d = (i + 1) * n_lon + j, (i + 1) * n_lon + j2
    band = np.stack([np.stack([a, b, d], -1), np.stack([a, d, c], -1)], 2).reshape(-1, 3)
    jj = np.arange(n_lon)
    jj2 = (jj + 1) % n_lon
    top = (nr - 1) * n_lon
    south = np.stack([np.full(n_lon, S), jj2, jj], -1)
    north = np.stack([np.full(n_lon, N), top + jj, top + jj2], -1)
    caps = np.stack([south, north], 1).reshape(-1, 3)
    faces = np.concatenate([band, caps])
    faces = np.asarray(faces, np.int64)
    return verts, _orient_outward(verts, faces)


def _orient_outward(verts, faces):
    a, b, c = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum()
    if vol < 0:
        faces = faces[:, [0, 2, 1]]
    return faces


def vertex_normals(verts, faces):
    a, b, c = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    fn = np.cross(b - a, c - a)
    vn = np.zeros_like(verts)
    for k in range(3):
        np.add.at(vn, faces[:, k], fn)
    return vn / np.maximum(np.linalg.norm(vn, axis=1, keepdims=True), 1e-30)


class Perlin3:
    """Improved Perlin gradient noise with a seeded permutation table."""

    _G = np.array([[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1],
                   [1, 0, -1], [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1],
                   [1, 1, 0], [0, -1, 1], [-1, 1, 0], [0, -1, -1]], dtype=np.float64)

    def __init__(self, seed: int):
        p = np.random.default_rng(seed).permutation(256)
        self.p = np.concatenate([p, p])

    def __call__(self, pts: np.ndarray) -> np.ndarray:
        pi = np.floor(pts).astype(np.int64)
        pf = pts - pi
        pi &= 255
        fade = pf * pf * pf * (pf * (pf * 6 - 15) + 10)
        p = self.p
        out = np.zeros(len(pts))
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    h = p[p[p[pi[:, 0] + dx] + pi[:, 1] + dy] + pi[:, 2] + dz] & 15
                    g = self._G[h]
                    rel = pf - np.array([dx, dy, dz])
                    dotv = (g * rel).sum(1)
                    w = ((fade[:, 0] if dx else 1 - fade[:, 0]) *
                         (fade[:, 1] if dy else 1 - fade[:, 1]) *
                         (fade[:, 2] if dz else 1 - fade[:, 2]))
                    out += w * dotv
        return out


def room(half_w=2.0, floor_y=-1.0, ceil_y=2.0, back_z=4.0, n_a=16, n_b=8):
    """Floor y = floor_y, side walls x = +-half_w, back wall z = back_z, each an
    n_a x n_b grid of quads (2 n_a n_b triangles per surface)."""
    parts = []

    def grid(p0, ua, ub):
        ia, ib = np.meshgrid(np.arange(n_a + 1), np.arange(n_b + 1), indexing="ij")
        pts = p0 + ia[..., None] / n_a * ua + ib[..., None] / n_b * ub
        pts = pts.reshape(-1, 3)
        f = []
        for i in range(n_a):
            for j in range(n_b):
                a = i * (n_b + 1) + j
                b = (i + 1) * (n_b + 1) + j
                f += [[a, b, b + 1], [a, b + 1, a + 1]]
        return pts, np.asarray(f, np.int64)

    h = ceil_y - floor_y
    parts.append(grid(np.array([-half_w, floor_y, 0.0]), np.array([2 * half_w, 0, 0]), np.array([0, 0, back_z])))
    parts.append(grid(np.array([-half_w, floor_y, 0.0]), np.array([0, 0, back_z]), np.array([0, h, 0])))
    parts.append(grid(np.array([half_w, floor_y, 0.0]), np.array([0, 0, back_z]), np.array([0, h, 0])))
    parts.append(grid(np.array([-half_w, floor_y, back_z]), np.array([2 * half_w, 0, 0]), np.array([0, h, 0])))
    return _concat(parts)


def cube(center, half: float):
    """Axis-aligned cube, 12 triangles."""
    v = np.array([[x, y, z] for x in (-half, half) for y in (-half, half) for z in (-half, half)], float)
    f = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
                  [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]])
    return v + np.asarray(center, float), f


def _concat(parts):
    vs, fs, off = [], [], 0
    for v, f in parts:
        vs.append(v)
        fs.append(f + off)
        off += len(v)
    return np.concatenate(vs), np.concatenate(fs)


def _rot_from_to(a, w):
    """Rotation taking unit vector a to unit vector w with a fixed roll."""
    a = a / np.linalg.norm(a)
    w = w / np.linalg.norm(w)
    a2 = np.cross(a, [0.0, 1.0, 0.0]) if abs(a[1]) < 0.9 else np.cross(a, [1.0, 0.0, 0.0])
    a2 /= np.linalg.norm(a2)
    w2 = np.cross(w, [0.0, 1.0, 0.0]) if abs(w[1]) < 0.9 else np.cross(w, [1.0, 0.0, 0.0])
    w2 /= np.linalg.norm(w2)
    Ba = np.stack([a, a2, np.cross(a, a2)], 1)
    Bw = np.stack([w, w2, np.cross(w, w2)], 1)
    return Bw @ Ba.T


def trihedral(leg: float, subdivide: bool = True):
    """Corner reflector: three mutually perpendicular right-isosceles faces with
    legs `leg` meeting at the origin, opening toward +(1,1,1).  With subdivide,
    each face is split 1->4 at its edge midpoints (12 right-isosceles triangles)."""
    L = leg
    o, X, Y, Z = np.zeros(3), np.array([L, 0, 0.0]), np.array([0, L, 0.0]), np.array([0, 0, L])
    big = [(o, X, Y), (o, Z, X), (o, Y, Z)]
    tris = []
    for a, b, c in big:
        if subdivide:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            tris += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        else:
            tris.append((a, b, c))
    pts = np.array([p for t in tris for p in t])
    faces = np.arange(len(pts)).reshape(-1, 3)
    return _dedupe(pts, faces)


def plate(size: float, z: float):
    h = size / 2.0
    v = np.array([[-h, -h, z], [h, -h, z], [h, h, z], [-h, h, z]])
    f = np.array([[0, 2, 1], [0, 3, 2]])   # normal toward -z (facing the radar)
    return v, f


# --------------------------------------------------------------------------- configs
def trihedral_plate(with_trihedral: bool = True, with_plate: bool = True) -> Scene:
    """Corner reflector (0.1 m legs, apex 1.0 m at azimuth -9 deg, axis pointing
    at the radar) plus a 0.2 x 0.2 m plate on boresight at 1.5 m; 64 x 64 rays
    over a +-15 deg tangent grid, 3 bounces; 1 TX, 4 RX at lambda/2; one
    77 GHz chirp, 60 MHz/us, 256 samples at 10 MHz."""
    parts = []
    if with_trihedral:
        tv, tf = trihedral(0.1)
        az = math.radians(-9.0)
        apex = np.array([math.sin(az), 0.0, math.cos(az)]) * 1.0
        R = _rot_from_to(np.ones(3) / math.sqrt(3.0), -apex / np.linalg.norm(apex))
        parts.append((tv @ R.T + apex, tf))
    if with_plate:
        parts.append(plate(0.2, 1.5))
    v, f = _concat(parts)
    return Scene("trihedral_plate", v.astype(np.float32), f.astype(np.int32),
                 default_radar(1, 4), Chirp(n_chirps=1), Grid())


def trihedral_apex() -> np.ndarray:
    az = math.radians(-9.0)
    return np.array([math.sin(az), 0.0, math.cos(az)])


def icosphere_scene(level: int = 5, radius: float = 0.2, dist: float = 1.5,
                    jitter: float = 2e-3, seed: int = 2, n_rays: int = 512,
                    n_chirps: int = 64, bounces: int = 3) -> Scene:
    """Icosphere of `level` subdivisions (level 5: 20480 triangles), radius
    0.2 m centred 1.5 m on boresight, iid Gaussian vertex jitter; 3TX x 4RX."""
    v, f = icosphere(level)
    v = v * radius + np.array([0.0, 0.0, dist])
    if jitter > 0:
        v = v + np.random.default_rng(seed).normal(0.0, jitter, v.shape)
    th = fov_tan(radius + 4 * jitter, dist)
    return Scene(f"icosphere_l{level}", v.astype(np.float32), f.astype(np.int32),
                 default_radar(3, 4, vel=(0.0, 0.0, 1.0)), Chirp(n_chirps=n_chirps),
                 Grid(n_rays, n_rays, th, th, bounces))


def superquadric_object(seed: int, n_lon: int, n_lat: int, axes, center,
                        noise_amp: float = 0.0, noise_cycles: float = 4.0,
                        e_range=(0.3, 2.0)):
    rng = np.random.default_rng(seed)
    e1, e2 = rng.uniform(*e_range, size=2)
    v, f = superquadric(n_lon, n_lat, axes, float(e1), float(e2))
    if noise_amp > 0:
        size = 2.0 * max(axes)
        pn = Perlin3(seed)
        n = vertex_normals(v, f)
        disp = pn(v * (noise_cycles / size) + 0.5)
        v = v + n * (noise_amp * disp)[:, None]
    return v + np.asarray(center, float), f


def clutter_scene(seed: int = 3, n_rays: int = 2048, n_chirps: int = 128,
                  bounces: int = 4, n_lon: int = 224, n_lat: int = 113) -> Scene:
    """Superquadric (exponents U(0.3, 2), half-axes 0.4/0.3/0.3 m, Perlin
    displacement of 2 % of its size, ~50k triangles) at 2 m, inside a room of
    a floor and three walls (1024 triangles); +-20 deg, 4 bounces, 12 virtual
    antennas x 128 chirps x 256 samples."""
    axes = (0.4, 0.3, 0.3)
    ov, of = superquadric_object(seed, n_lon, n_lat, axes, (0.0, 0.0, 2.0),
                                 noise_amp=0.02 * 0.4)
    rv, rf = room()
    v, f = _concat([(ov, of), (rv, rf)])
    th = math.tan(math.radians(20.0))
    return Scene("clutter_50k", v.astype(np.float32), f.astype(np.int32),
                 default_radar(3, 4, vel=(0.0, 0.0, 1.0)), Chirp(n_chirps=n_chirps),
                 Grid(n_rays, n_rays, th, th, bounces))


def imaging_scene(n_rays: int = 512, n_chirps: int = 16, n_samples: int = 256, seed: int = 5,
                  n_tx: int = 20, n_rx: int = 20, bounces: int = 2) -> Scene:
    """Planar-array imaging workload: 20 TX x 20 RX (400 virtual antennas,
    lambda/2 grid) at 62 GHz with a 7 GHz sweep in the ADC window (256 samples
    at 10 MHz, 2.1 cm range bins, 5.5 m unambiguous), 16 chirps; two
    superquadrics (~10k triangles each) and a corner reflector 1-2 m out,
    +-25 deg, 2 bounces, scene velocity 0.5 m/s."""
    a, fa = superquadric_object(seed, 100, 51, (0.15, 0.2, 0.12), (-0.35, 0.1, 1.4))
    b, fb = superquadric_object(seed + 1, 100, 51, (0.2, 0.12, 0.18), (0.4, -0.15, 1.9))
    tv, tf = trihedral(0.12)
    apex = np.array([0.05, 0.35, 1.2])
    R = _rot_from_to(np.ones(3) / math.sqrt(3.0), -apex / np.linalg.norm(apex))
    v, f = _concat([(a, fa), (b, fb), (tv @ R.T + apex, tf)])
    th = math.tan(math.radians(25.0))
    ch = Chirp(fc=62e9, slope=7e9 / (n_samples / 10e6), fs=10e6, t_chirp=40e-6, n_samples=n_samples,
               n_chirps=n_chirps)
    return Scene("imaging_400", v.astype(np.float32), f.astype(np.int32),
                 planar_radar(n_tx, n_rx, 62e9, vel=(0.0, 0.0, 0.5)), ch, Grid(n_rays, n_rays, th, th, bounces))


def recon_scenes(seed: int = 4, n_rays: int = 1024, n_chirps: int = 64):
    """Reconstruction workload: start = geodesic sphere (freq 22, 9680
    triangles) of radius 0.2 m at 1.5 m; target = superquadric of ~10k
    triangles with half-axes U(0.15, 0.25) m at the same centre."""
    gv, gf = geodesic_sphere(22)
    centre = np.array([0.0, 0.0, 1.5])
    start_v = gv * 0.2 + centre
    rng = np.random.default_rng(seed)
    axes = tuple(rng.uniform(0.15, 0.25, size=3))
    tv, tf = superquadric_object(seed, 100, 51, axes, centre)
    th = fov_tan(0.25 * 1.05, 1.5)
    radar = default_radar(3, 4, vel=(0.0, 0.0, 1.0))
    grid = Grid(n_rays, n_rays, th, th, 3)
    start = Scene("recon_start", start_v.astype(np.float32), gf.astype(np.int32), radar,
                  Chirp(n_chirps=n_chirps), grid)
    target = Scene("recon_target", tv.astype(np.float32), tf.astype(np.int32), radar,
                   Chirp(n_chirps=n_chirps), grid)
    return start, target


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float
    scene: Scene
    backward: bool
    target: Optional[np.ndarray] = None     # filled in by the caller for backward requests


def serving_requests(n: int = 512, qps: float = 10.0, seed: int = 5,
                     grids=(256, 512, 1024, 2048), nf_range=(1000, 200000),
                     chirps=(32, 64, 128)) -> List[Request]:
    """Poisson stream of simulation requests: superquadric meshes with
    log-uniform triangle counts, random size and distance, ray grids, bounce
    counts, TX counts and chirp counts; 30 % also ask for the backward pass."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / qps)
        r = np.random.default_rng(5000 + i)
        nf = math.exp(r.uniform(math.log(nf_range[0]), math.log(nf_range[1])))
        nlat = max(3, int(round(math.sqrt(nf / 4.0)))) + 1
        nlon = 2 * (nlat - 1)
        size = r.uniform(0.15, 0.5)
        dist = r.uniform(1.0, 3.0)
        axes = tuple(size * r.uniform(0.6, 1.0, size=3))
        v, f = superquadric_object(int(r.integers(1 << 30)), nlon, nlat, axes, (0.0, 0.0, dist))
        g = int(r.choice(grids))
        K = int(r.integers(2, 5))
        ntx = int(r.integers(1, 4))
        C = int(r.choice(chirps))
        th = fov_tan(max(axes) * 1.05, dist)
        sc = Scene(f"req{i}", v.astype(np.float32), f.astype(np.int32),
                   default_radar(ntx, 4, vel=(0.0, 0.0, 1.0)), Chirp(n_chirps=C),
                   Grid(g, g, th, th, K))
        out.append(Request(i, t, sc, bool(r.uniform() < 0.3)))
    return out


def jitter(scene: Scene, sigma: float, seed: int) -> Scene:
    v = scene.verts.astype(np.float64)
    v = v + np.random.default_rng(seed).normal(0.0, sigma, v.shape)
    return scene.with_verts(v)


def room_scene(n_rays: int = 48, boxes: bool = True, shadow: bool = True, n_chirps: int = 2,
               n_samples: int = 16) -> Scene:
    """Radar at the open front of a room (floor, side and back walls of 8 x 4
    quads each) with two boxes inside that hide parts of the walls from it;
    4 bounces over a wide (+-42 x +-35 deg) grid, 1 TX x 2 RX.  A scene rich in
    returns whose way back to the radar is blocked."""
    parts = [room(n_a=8, n_b=4)]
    if boxes:
        parts += [cube([0.6, -0.5, 2.2], 0.45), cube([-1.0, 0.2, 1.4], 0.25)]
    v, f = _concat(parts)
    return Scene("room_boxes" if boxes else "room", v.astype(np.float32), f.astype(np.int32),
                 default_radar(1, 2), Chirp(n_chirps=n_chirps, n_samples=n_samples),
                 Grid(n_rays, n_rays, 0.9, 0.7, 4, shadow=shadow))


def single_triangle(z: float = 1.0, size: float = 0.1) -> Scene:
    v = np.array([[-size, -size, z], [size, -size, z], [0.0, size, z]], np.float32)
    f = np.array([[0, 1, 2]], np.int32)
    return Scene("triangle", v, f, default_radar(1, 4), Chirp(), Grid(16, 16, 0.12, 0.12, 2))
