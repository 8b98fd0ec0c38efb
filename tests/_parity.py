"""Helpers shared by the GPU parity tests (HIP path vs FP64 oracle)."""
from __future__ import annotations

import sys
import time

import numpy as np

FLAG_MASK = 0xFF
GEOM_FLAGS = 0x1F      # edge, tie, graze, t_min, parent (not the occlusion bit)


def log(msg: str):
    print(f"[parity {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.reshape(-1))
    return float(np.linalg.norm((a - b).reshape(-1)) / (den if den > 0 else 1.0))


def device_hits_from_oracle(tr, device="cuda"):
    """Upload the oracle's hit records into the library's hit layout (the
    oracle's values are inputs to the HIP path here)."""
    import torch
    from paper_2311_13182_amd.sbr import Hits
    return Hits(torch.as_tensor(tr["tri"].astype(np.int32), device=device).contiguous(),
                torch.as_tensor(tr["t"].astype(np.float32), device=device).contiguous(),
                torch.as_tensor(tr["b1"].astype(np.float32), device=device).contiguous(),
                torch.as_tensor(tr["b2"].astype(np.float32), device=device).contiguous(),
                torch.as_tensor(tr["flags"].astype(np.uint8), device=device).contiguous())


def scatter_sampled_hits(tr_sub, rays, K, R):
    """Full-grid hit arrays in which only the sampled rays have hits."""
    full = {"tri": np.full((K, R), -1, np.int32), "t": np.zeros((K, R)), "b1": np.zeros((K, R)),
            "b2": np.zeros((K, R)), "flags": np.zeros((K, R), np.uint8)}
    for k in ("tri", "t", "b1", "b2", "flags"):
        full[k][:, rays] = tr_sub[k]
    return full


def compare_trace(gpu, orc, rays=None, L_prev=None):
    """IDs bit-exact except rays with a geometric flag (either side); t within
    1e-5 (L_{k-1} + t) at the first bounce, and within 1e-5 (L_{k-1} + t) /
    cos(theta_k) at later ones, whose FP32 origin and direction errors the
    ray-plane intersection magnifies by 1 / cos(theta_k) (theta_k the
    incidence angle, from the oracle).  Returns (n_checked, n_flagged)."""
    tri_g = gpu["tri"] if rays is None else gpu["tri"][:, rays]
    t_g = gpu["t"] if rays is None else gpu["t"][:, rays]
    fl_g = gpu["flags"] if rays is None else gpu["flags"][:, rays]
    K, n = orc["tri"].shape
    flagged = ((fl_g & GEOM_FLAGS) != 0) | ((orc["flags"] & GEOM_FLAGS) != 0)
    # once a bounce is flagged on either side, later bounces are not comparable
    anc = np.logical_or.accumulate(flagged, axis=0)
    ok = ~anc
    mism = ok & (tri_g != orc["tri"])
    if mism.any():
        k, i = np.argwhere(mism)[0]
        raise AssertionError(f"hit id mismatch at bounce {k} ray {i if rays is None else rays[i]}: "
                             f"gpu {tri_g[k, i]} oracle {orc['tri'][k, i]} (t {t_g[k, i]} / {orc['t'][k, i]})")
    Lp = np.zeros(n)
    for k in range(K):
        m = ok[k] & (orc["tri"][k] >= 0)
        err = np.abs(t_g[k][m] - orc["t"][k][m])
        tol = 1e-5 * (Lp[m] + orc["t"][k][m])
        if k > 0 and "cos" in orc and m.any():
            lit = err / tol
            w = int(np.argmax(lit))
            log(f"  bounce {k}: worst t error {lit[w]:.2f} x the uncorrected tolerance, at cos {orc['cos'][k][m][w]:.3e}")
            tol = tol / np.maximum(orc["cos"][k][m], 1e-6)
        if not (err <= tol).all():
            w = int(np.argmax(err / tol))
            cs = orc["cos"][k][m][w] if "cos" in orc else float("nan")
            raise AssertionError(f"t mismatch at bounce {k}: err {err[w]:.3e} > tol {tol[w]:.3e} "
                                 f"(t {orc['t'][k][m][w]:.6f}, L_prev {Lp[m][w]:.4f}, cos {cs:.3e})")
        Lp = Lp + np.where(orc["tri"][k] >= 0, orc["t"][k], 0.0)
    return int((ok & (orc["tri"] >= 0)).sum()), int(anc.sum())


def union_flags(gpu_flags, orc_flags):
    """The comparison mask of a record-by-record check: a record flagged on
    either side (either side's hit could be the other's neighbour) is dropped
    on both sides, with the later bounces of its ray."""
    return (np.asarray(gpu_flags, np.uint8) | np.asarray(orc_flags, np.uint8)).astype(np.uint8)


def fd_coords_local(orc, sc, tri, flags, target, coords, h=1e-9):
    """Central differences of the oracle's IF loss for single vertex
    coordinates with the hit sequences frozen, re-evaluating only the rays
    whose hit faces touch the moved vertex: Eq. 8 is a sum over paths, and the
    other rays' paths do not depend on that vertex."""
    base_p = orc.paths(sc, tri, flags)
    S_base = orc.synth(sc, base_p)
    v0 = sc.verts.astype(np.float64)
    out = np.zeros(len(coords))
    for i, c in enumerate(coords):
        vi, ax = int(c) // 3, int(c) % 3
        faces = np.flatnonzero((sc.faces == vi).any(axis=1))
        rays = np.flatnonzero(np.isin(tri, faces).any(axis=0))
        if len(rays) == 0:
            continue
        sub_tri = np.ascontiguousarray(tri[:, rays])
        sub_fl = np.ascontiguousarray(flags[:, rays])
        base = orc.synth(sc, orc.paths(sc, sub_tri, sub_fl, rays=rays))
        Ls = []
        for sgn in (+1.0, -1.0):
            v = v0.copy()
            v[vi, ax] += sgn * h
            pert = orc.synth(sc, orc.paths(sc, sub_tri, sub_fl, rays=rays, verts64=v))
            Ls.append(orc.if_loss(S_base - base + pert, target))
        out[i] = (Ls[0] - Ls[1]) / (2.0 * h)
    return out
