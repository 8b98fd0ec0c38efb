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
