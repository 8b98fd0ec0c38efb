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
    1e-5 (L_{k-1} + t).  Returns (n_checked, n_flagged)."""
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
        assert (err <= tol).all(), f"t mismatch at bounce {k}: max err {err.max()}"
        Lp = Lp + np.where(orc["tri"][k] >= 0, orc["t"][k], 0.0)
    return int((ok & (orc["tri"] >= 0)).sum()), int(anc.sum())
