"""Pins of the oracle's reparameterised estimator (Sec. 3.2.1, Eqs. 6-7): the
transform T attaches each sample to its first hit (fixed barycentrics on the
moving triangle) and the cell weight carries |det J_T|.  CPU only.

- summed attached weights == closed-form solid angle of a triangle (Van
  Oosterom-Strackee), and their derivative == the closed form's;
- at the unperturbed scene the attached estimator is the fixed one;
- loose: its frozen-topology derivative == the derivative of the re-traced
  estimator on a dense grid (visibility changes included), while the
  fixed-direction (pathwise) derivative misses the silhouette term.
"""
import dataclasses
import math

import numpy as np

from paper_2311_13182_amd import scenes as S


def solid_angle(tri, o):
    """Van Oosterom & Strackee (1983): solid angle of triangle tri [3][3] seen from o."""
    R = np.asarray(tri, float) - np.asarray(o, float)
    r = np.linalg.norm(R, axis=1)
    num = abs(np.dot(R[0], np.cross(R[1], R[2])))
    den = r[0] * r[1] * r[2] + np.dot(R[0], R[1]) * r[2] + np.dot(R[0], R[2]) * r[1] + np.dot(R[1], R[2]) * r[0]
    return 2.0 * math.atan2(num, den)


def _triangle_scene(n):
    v = np.array([[-0.08, -0.06, 1.0], [0.09, -0.05, 1.04], [0.01, 0.08, 0.97]], np.float32)
    f = np.array([[0, 1, 2]], np.int32)
    sc = S.Scene("tri", v, f, S.default_radar(1, 2), S.Chirp(n_chirps=2, n_samples=16),
                 S.Grid(n, n, 0.11, 0.11, 1))
    return sc


def test_attached_weights_sum_to_solid_angle_and_its_derivative(orc):
    sc = _triangle_scene(400)
    tr = orc.trace(sc)
    att = orc.attach(sc, tr["tri"])
    v0 = sc.verts.astype(np.float64)
    o = np.zeros(3)
    p0 = orc.paths(sc, tr["tri"], tr["flags"], drop=False, att=att)
    # at theta_0 the weights are the cells' solid angles: their sum is the
    # grid's coverage of the triangle (edge cells make the O(1/n) error)
    assert abs(p0["weight"].sum() / solid_angle(v0, o) - 1.0) < 5e-3
    rng = np.random.default_rng(3)
    for trial in range(4):
        w = rng.normal(size=v0.shape)
        if trial == 0:
            w = np.zeros_like(v0)
            w[:, 2] = 1.0          # whole triangle toward / away from the radar
        w /= np.linalg.norm(w)
        h = 1e-5
        W = []
        for sg in (1.0, -1.0):
            p = orc.paths(sc, tr["tri"], tr["flags"], drop=False, verts64=v0 + sg * h * w, att=att)
            W.append(p["weight"].sum())
        dW = (W[0] - W[1]) / (2 * h)
        dO = (solid_angle(v0 + h * w, o) - solid_angle(v0 - h * w, o)) / (2 * h)
        assert abs(dW - dO) <= 1e-2 * abs(dO), (trial, dW, dO)


def test_attached_equals_fixed_at_theta0(orc):
    sc = S.trihedral_plate()
    tr = orc.trace(sc)
    att = orc.attach(sc, tr["tri"])
    a = orc.paths(sc, tr["tri"], tr["flags"])
    b = orc.paths(sc, tr["tri"], tr["flags"], att=att)
    assert len(a["amp"]) == len(b["amp"]) > 0
    assert np.allclose(b["amp"], a["amp"], rtol=1e-10, atol=0)
    assert np.allclose(b["tau"], a["tau"], rtol=1e-12, atol=0)
    assert np.allclose(b["taudot"], a["taudot"], rtol=1e-10, atol=1e-30)


def _plate_scene(n):
    """0.2 m square plate 1 m out, turned 17 deg about boresight (no edge
    parallel to the ray grid), 2 antennas, 2 chirps x 32 samples."""
    v, f = S.plate(0.2, 1.0)
    c, s = math.cos(math.radians(17.0)), math.sin(math.radians(17.0))
    R = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    v = v @ R.T + np.array([0.01, -0.02, 0.0])
    return S.Scene("plate", v.astype(np.float32), f.astype(np.int32), S.default_radar(1, 2),
                   S.Chirp(n_chirps=2, n_samples=32), S.Grid(n, n, 0.16, 0.16, 1))


def test_attached_derivative_matches_dense_retraced_grid(orc):
    sc = _plate_scene(640)
    tr = orc.trace(sc)
    att = orc.attach(sc, tr["tri"])
    # target: the plate moved 3 mm sideways and 1 mm out
    tsc = dataclasses.replace(sc, verts=(sc.verts + np.array([0.003, 0.0, 0.001], np.float32)))
    tgt, _, _ = orc.forward(tsc, drop=False)
    w_shift = np.zeros((sc.nv, 3))
    w_shift[:, 0] = 1.0                     # in-plane translation: only silhouettes move
    w_shift /= np.linalg.norm(w_shift)
    w_corner = np.zeros((sc.nv, 3))
    w_corner[2] = [0.6, 0.8, 0.0]           # one corner moves in-plane: area and silhouette
    for w in (w_shift, w_corner):
        ref = orc.fd_retraced(sc, tgt, w, h=1e-3)
        an = orc.fd_directional(sc, tr["tri"], tr["flags"], tgt, w, h=1e-7, drop=False, att=att)
        pw = orc.fd_directional(sc, tr["tri"], tr["flags"], tgt, w, h=1e-7, drop=False)
        assert abs(an - ref) <= 0.03 * abs(ref), (an, ref)   # 0.7 % at 640^2, 3-4 % at 320^2
        assert abs(pw - ref) > 0.5 * abs(ref), (pw, ref)


# ----------------------------------------------------------------------------- occlusion-tested returns
def _room_scene(with_box, n=48):
    return S.room_scene(n_rays=n, boxes=with_box)


def _segment_blocked(v, f, x, O, self_id, t_min):
    """Independent NumPy segment test against every triangle but self_id."""
    s = O - x
    D = np.linalg.norm(s)
    s = s / D
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    e1, e2 = b - a, c - a
    p = np.cross(s, e2)
    det = np.einsum("ij,ij->i", e1, p)
    ok = det != 0
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    tv = x - a
    u = np.einsum("ij,ij->i", tv, p) * inv
    q = np.cross(tv, e1)
    w = (q @ s) * inv
    t = np.einsum("ij,ij->i", e2, q) * inv
    hit = ok & (u >= 0) & (w >= 0) & (u + w <= 1) & (t > t_min) & (t < D - t_min)
    hit[self_id] = False
    return bool(hit.any())


def test_shadow_convex_room_never_occluded(orc):
    sc = _room_scene(False)
    tr = orc.trace(sc)
    hits = tr["tri"] >= 0
    assert hits[1:].sum() > 1000                       # plenty of later bounces
    assert not (tr["flags"] & orc.F_OCCLUDED).any()


def test_shadow_bits_vs_independent_brute_force(orc):
    sc = _room_scene(True)
    tr = orc.trace(sc)
    v = sc.verts.astype(np.float64)
    f = sc.faces
    occ = (tr["flags"] & orc.F_OCCLUDED) != 0
    assert not occ[0].any()                            # a first hit's return retraces its ray
    K, n = tr["tri"].shape
    checked = disagree = 0
    for k in range(1, K):
        for i in np.nonzero(tr["tri"][k] >= 0)[0]:
            if tr["shadow_edge"][k, i]:
                continue
            fid = tr["tri"][k, i]
            a, b, c = v[f[fid, 0]], v[f[fid, 1]], v[f[fid, 2]]
            x = a + tr["b1"][k, i] * (b - a) + tr["b2"][k, i] * (c - a)
            want = _segment_blocked(v, f, x, np.zeros(3), fid, sc.grid.t_min)
            checked += 1
            disagree += int(want != occ[k, i])
    assert checked > 1000 and occ.sum() > 100
    assert disagree == 0
    # occlusion is not inherited: a later bounce after an occluded one can return
    later = occ[1:-1] & (tr["tri"][2:] >= 0) & ~occ[2:]
    assert later.any()
    own = tr["flags"] & ~np.uint8(orc.F_OCCLUDED | orc.F_PARENT)       # geometric flags of each bounce
    inherited = np.logical_or.accumulate(own != 0, axis=0)
    parent = (tr["flags"] & orc.F_PARENT) != 0
    hit = tr["tri"] >= 0
    assert np.array_equal(parent[1:][hit[1:]], inherited[:-1][hit[1:]])


def test_exit_only_keeps_last_hit_of_each_ray(orc):
    sc = _room_scene(True, n=24)
    tr = orc.trace(sc)
    full = orc.paths(sc, tr["tri"], tr["flags"], drop=False)
    ex = orc.paths(sc, tr["tri"], tr["flags"], drop=False, exit_only=True)
    nb = (tr["tri"] >= 0).sum(axis=0)                 # hits per ray
    last = nb - 1
    occ_last = np.array([tr["flags"][last[i], i] & orc.F_OCCLUDED if nb[i] else 0 for i in range(len(nb))])
    want = np.nonzero((nb > 0) & (occ_last == 0))[0]
    assert np.array_equal(ex["ray"], want)
    assert np.array_equal(ex["k"], nb[want])
    # the same records as in the full model
    key = {(r, k): j for j, (r, k) in enumerate(zip(full["ray"], full["k"]))}
    idx = np.array([key[(r, k)] for r, k in zip(ex["ray"], ex["k"])])
    assert np.array_equal(ex["amp"], full["amp"][idx]) and np.array_equal(ex["tau"], full["tau"][idx])
