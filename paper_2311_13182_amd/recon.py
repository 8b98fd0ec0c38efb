"""Gradient-based mesh reconstruction from a radar IF cube (paper Sec. 3.4,
Eqs. 14-15; Fig. 1's loop: simulate, compare, backpropagate, update).

Parameters are per-vertex offsets of a start mesh.  The gradient is the
pathwise one of the fixed-grid estimator being minimised; `attached=True`
takes the reparameterised one of Eqs. 6-7 instead (the derivative of the
underlying integral, silhouettes included), which agrees with the former only
once the ray grid resolves the phase across the surface.
The objective is either the spatial multi-antenna loss of Eq. (16) -- MSE
between the images |T(S)|^2 of the simulated and the target signal, T =
range/Doppler/angle DFTs -- or the plain IF-domain MSE, each normalised by
its target, plus a uniform-Laplacian smoothness term on the offsets; the
optimiser is Adam.  The simulator runs in libsbr (BVH refit every step, full
rebuild every `rebuild_every` steps); torch holds the parameters, runs Adam
and the regulariser.
"""
from __future__ import annotations

import dataclasses
import json
import math
import time
from typing import List, Optional

import numpy as np
import torch

from . import scenes as S
from .autograd import HeatmapLoss, IFLoss, RadarCubeFunction, SBRFunction, box_pose, rigid_pose
from .sbr import Simulator


def uniform_laplacian(offsets: torch.Tensor, edges: torch.Tensor, deg: torch.Tensor) -> torch.Tensor:
    """sum_i |d_i - mean_{j in N(i)} d_j|^2 for offsets d [nv,3]."""
    acc = torch.zeros_like(offsets)
    acc.index_add_(0, edges[:, 0], offsets[edges[:, 1]])
    mean = acc / deg[:, None]
    return ((offsets - mean) ** 2).sum()


def mesh_edges(faces: np.ndarray, nv: int):
    e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]])
    e = np.unique(e, axis=0)
    deg = np.bincount(e[:, 0], minlength=nv).astype(np.float32)
    return e, np.maximum(deg, 1.0)


def area_samples(verts: np.ndarray, faces: np.ndarray, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a, b, c = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    f = rng.choice(len(faces), size=n, p=area / area.sum())
    u, v = rng.uniform(size=n), rng.uniform(size=n)
    flip = u + v > 1
    u[flip], v[flip] = 1 - u[flip], 1 - v[flip]
    return a[f] + u[:, None] * (b[f] - a[f]) + v[:, None] * (c[f] - a[f])


def chamfer(va, fa, vb, fb, n=10000, seed=44, device="cuda") -> float:
    """Symmetric Chamfer distance: mean squared nearest-neighbour distance
    between n area-uniform samples of each mesh, both directions, summed."""
    pa = torch.as_tensor(area_samples(np.asarray(va, np.float64), fa, n, seed), device=device)
    pb = torch.as_tensor(area_samples(np.asarray(vb, np.float64), fb, n, seed + 1), device=device)

    def one(p, q):
        best = []
        for i in range(0, len(p), 2048):
            best.append(torch.cdist(p[i:i + 2048], q).min(dim=1).values ** 2)
        return torch.cat(best).mean()

    return float(one(pa, pb) + one(pb, pa))


@dataclasses.dataclass
class ReconResult:
    losses: List[float]
    step_ms: List[float]
    chamfer_start: float
    chamfer_final: float
    lam: float
    verts: np.ndarray


def reconstruct(start: S.Scene, target: S.Scene, steps: int = 200, lr: float = 1e-3,
                rebuild_every: int = 20, device="cuda", log_every: int = 0, objective: str = "heatmap",
                lam_scale: float = 0.1, checkpoint: Optional[str] = None, resume: Optional[str] = None,
                attached: bool = False, mc_seed: Optional[int] = None) -> ReconResult:
    dev = torch.device(device)
    sim = Simulator(start, dev)
    # target signal (untimed)
    tsim = Simulator(target, dev)
    tcube = tsim.forward().clone()
    del tsim
    if objective not in ("heatmap", "if"):
        raise ValueError(f"objective must be 'heatmap' or 'if', not {objective!r}")
    if objective == "heatmap":
        tgt = (sim.radar_cube(tcube).abs() ** 2).contiguous()
        tnorm = float((tgt ** 2).mean().item())
    else:
        tgt = tcube
        tnorm = float((tgt.abs() ** 2).sum().item())

    def data_term(cube):
        if objective == "heatmap":
            return HeatmapLoss.apply(RadarCubeFunction.apply(cube, sim, 0), tgt, sim, 1.0 / tnorm)
        return IFLoss.apply(cube, tgt, sim, 1.0 / tnorm)

    base = torch.as_tensor(start.verts, dtype=torch.float32, device=dev)
    offsets = torch.zeros_like(base, requires_grad=True)
    opt = torch.optim.Adam([offsets], lr=lr)
    e, deg = mesh_edges(start.faces.astype(np.int64), start.nv)
    edges = torch.as_tensor(e, device=dev)
    degt = torch.as_tensor(deg, device=dev)
    # lambda: a 1 mm iid roughness of the offsets costs lam_scale (default 10 %)
    # of the initial data term
    with torch.no_grad():
        d0 = float(data_term(SBRFunction.apply(base, sim, False, attached)).item())
        rough = torch.as_tensor(np.random.default_rng(7).normal(0, 1e-3, size=start.verts.shape),
                                dtype=torch.float32, device=dev)
        lam = lam_scale * d0 / float(uniform_laplacian(rough, edges, degt).item())
    first = 0
    if resume:
        st = torch.load(resume, weights_only=True)
        offsets.data.copy_(st["offsets"])
        opt.load_state_dict(st["opt"])
        first = int(st["step"])
    losses, times = [], []
    sim.build()
    for it in range(first, steps):
        t0 = time.perf_counter()
        verts = base + offsets
        refit = (it % rebuild_every) != 0
        if mc_seed is not None:   # fresh stratified Monte Carlo samples each step (Eq. 4)
            sim.scene = sim.scene.with_grid(jitter_seed=(mc_seed << 20) + it)
        cube = SBRFunction.apply(verts, sim, refit, attached)
        data = data_term(cube)
        total = data + lam * uniform_laplacian(offsets, edges, degt)
        opt.zero_grad(set_to_none=True)
        total.backward()
        opt.step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        losses.append(float(total.item()))
        if log_every and (it % log_every == 0 or it == steps - 1):
            print(json.dumps({"step": it, "loss": losses[-1], "ms": round(times[-1], 2)}), flush=True)
        if checkpoint and (it + 1) % 20 == 0:
            torch.save({"offsets": offsets.detach().cpu(), "opt": opt.state_dict(), "step": it + 1}, checkpoint)
    final = (base + offsets).detach().cpu().numpy()
    c0 = chamfer(start.verts, start.faces, target.verts, target.faces, device=dev)
    c1 = chamfer(final, start.faces, target.verts, target.faces, device=dev)
    return ReconResult(losses, times, c0, c1, lam, final)


@dataclasses.dataclass
class PoseResult:
    losses: List[float]
    omega: np.ndarray
    trans: np.ndarray
    step_ms: List[float]


def fit_pose(scene: S.Scene, target_cube: torch.Tensor, steps: int = 100, lr: float = 2e-3,
             omega0=(0.0, 0.0, 0.0), trans0=(0.0, 0.0, 0.0), objective: str = "heatmap",
             device="cuda", rebuild_every: int = 20, attached: bool = False,
             mc_seed: Optional[int] = None) -> PoseResult:
    """Object pose from a radar IF cube (the object-transform parameterisation
    of Sec. 3.1 (i) driven by the loss of Eqs. 14/16): the mesh of `scene` is
    posed by exp([omega]x) about its centroid plus a translation, and Adam
    fits (omega, trans) so that its simulated signal matches `target_cube`."""
    dev = torch.device(device)
    sim = Simulator(scene, dev)
    if objective == "heatmap":
        tgt = (sim.radar_cube(target_cube).abs() ** 2).contiguous()
        tnorm = float((tgt ** 2).mean().item())
    elif objective == "if":
        tgt = target_cube
        tnorm = float((tgt.abs() ** 2).sum().item())
    else:
        raise ValueError(f"objective must be 'heatmap' or 'if', not {objective!r}")
    base = torch.as_tensor(scene.verts, dtype=torch.float32, device=dev)
    omega = torch.tensor(omega0, dtype=torch.float32, device=dev, requires_grad=True)
    trans = torch.tensor(trans0, dtype=torch.float32, device=dev, requires_grad=True)
    opt = torch.optim.Adam([omega, trans], lr=lr)
    losses, times = [], []
    for it in range(steps):
        t0 = time.perf_counter()
        if mc_seed is not None:   # fresh stratified Monte Carlo samples each step (Eq. 4)
            sim.scene = sim.scene.with_grid(jitter_seed=(mc_seed << 20) + it)
        cube = SBRFunction.apply(rigid_pose(base, omega, trans), sim, (it % rebuild_every) != 0, attached)
        if objective == "heatmap":
            loss = HeatmapLoss.apply(RadarCubeFunction.apply(cube, sim, 0), tgt, sim, 1.0 / tnorm)
        else:
            loss = IFLoss.apply(cube, tgt, sim, 1.0 / tnorm)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        losses.append(float(loss.item()))
    return PoseResult(losses, omega.detach().cpu().numpy(), trans.detach().cpu().numpy(), times)


@dataclasses.dataclass
class BoxResult:
    losses: List[float]
    log_scale: np.ndarray
    omega: np.ndarray
    trans: np.ndarray
    verts: np.ndarray
    chamfer_start: float
    chamfer_final: float
    step_ms: List[float]


def fit_box(start: S.Scene, target: S.Scene, steps: int = 150, lr: float = 3e-3, objective: str = "heatmap",
            device="cuda", window: int = 1, mc_seed: Optional[int] = None, attached: bool = False) -> BoxResult:
    """3D bounding-box case study (Sec. 3.1 (i)): the start mesh's transform --
    anisotropic scale, rotation, translation (`box_pose`) -- is fitted to the
    target's signal by Adam on the Eq. 16 loss (windowed radar cube)."""
    dev = torch.device(device)
    sim = Simulator(start, dev)
    tcube = Simulator(target, dev).forward().clone()
    if objective == "heatmap":
        tgt = (sim.radar_cube(tcube, window=window).abs() ** 2).contiguous()
        tnorm = float((tgt ** 2).mean().item())
    else:
        tgt, tnorm = tcube, float((tcube.abs() ** 2).sum().item())
    base = torch.as_tensor(start.verts, dtype=torch.float32, device=dev)
    ls = torch.zeros(3, device=dev, requires_grad=True)
    om = torch.zeros(3, device=dev, requires_grad=True)
    tr = torch.zeros(3, device=dev, requires_grad=True)
    opt = torch.optim.Adam([ls, om, tr], lr=lr)
    losses, times = [], []
    for it in range(steps):
        t0 = time.perf_counter()
        if mc_seed is not None:
            sim.scene = sim.scene.with_grid(jitter_seed=(mc_seed << 20) + it)
        cube = SBRFunction.apply(box_pose(base, ls, om, tr), sim, (it % 20) != 0, attached)
        if objective == "heatmap":
            loss = HeatmapLoss.apply(RadarCubeFunction.apply(cube, sim, window), tgt, sim, 1.0 / tnorm)
        else:
            loss = IFLoss.apply(cube, tgt, sim, 1.0 / tnorm)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        losses.append(float(loss.item()))
    final = box_pose(base, ls, om, tr).detach().cpu().numpy()
    c0 = chamfer(start.verts, start.faces, target.verts, target.faces, device=dev)
    c1 = chamfer(final, start.faces, target.verts, target.faces, device=dev)
    return BoxResult(losses, ls.detach().cpu().numpy(), om.detach().cpu().numpy(), tr.detach().cpu().numpy(),
                     final, c0, c1, times)


# --------------------------------------------------------------------------- point clouds (Fig. 1)
def chamfer_points(a: torch.Tensor, b: torch.Tensor) -> float:
    """Symmetric Chamfer distance between two point sets [n, 3] and [m, 3]:
    mean squared nearest-neighbour distance, both directions, summed."""
    if len(a) == 0 or len(b) == 0:
        return float("inf")
    d = torch.cdist(a.double(), b.double())
    return float((d.min(dim=1).values ** 2).mean() + (d.min(dim=0).values ** 2).mean())


def _kabsch(p: torch.Tensor, q: torch.Tensor):
    """Rotation R and translation t minimising sum |R p_i + t - q_i|^2."""
    pc, qc = p.mean(0), q.mean(0)
    H = (p - pc).T @ (q - qc)
    U, _, Vt = torch.linalg.svd(H)
    d = torch.sign(torch.linalg.det(Vt.T @ U.T))
    D = torch.diag(torch.stack([torch.ones_like(d), torch.ones_like(d), d]))
    R = Vt.T @ D @ U.T
    return R, qc - R @ pc


def register_rigid(src: torch.Tensor, dst: torch.Tensor, iters: int = 30, rotate: bool = True):
    """Rigid registration of point set src onto dst: centroid alignment, then
    point-to-point ICP (nearest neighbours + Kabsch).  Returns R [3,3], t [3]
    with dst ~ R src + t."""
    src, dst = src.double(), dst.double()
    R = torch.eye(3, dtype=torch.float64, device=src.device)
    t = dst.mean(0) - src.mean(0)
    if rotate:
        for _ in range(iters):
            cur = src @ R.T + t
            nn = torch.cdist(cur, dst).argmin(dim=1)
            R, t = _kabsch(src, dst[nn])
    return R, t


def rotation_to_axis_angle(R: torch.Tensor) -> torch.Tensor:
    c = ((torch.trace(R) - 1.0) / 2.0).clamp(-1.0, 1.0)
    th = torch.arccos(c)
    w = torch.stack([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    s = torch.sin(th)
    return w * (0.5 if float(th) < 1e-6 else float(th / (2.0 * s)))


@dataclasses.dataclass
class CloudFitResult:
    omega_init: np.ndarray
    trans_init: np.ndarray
    pose: PoseResult
    chamfer_cloud_start: float     # template cloud vs target cloud, before registration
    chamfer_cloud_init: float      # after point-cloud registration
    chamfer_cloud_final: float     # after the signal-domain fit
    n_target_points: int


def fit_from_point_cloud(template: S.Scene, target_cube: torch.Tensor, steps: int = 60, lr: float = 2e-3,
                         objective: str = "heatmap", device="cuda", pfa: float = 1e-4,
                         rotate: Optional[bool] = None, snr_db: Optional[float] = 20.0) -> CloudFitResult:
    """Fig. 1's loop from a radar measurement: the target signal is turned
    into a point cloud (radar cube, CA-CFAR, detections to points); the
    template mesh is registered to it (centroid + ICP of the template's own
    simulated cloud) to initialise its pose (Sec. 3.1, initialisation from
    point clouds by registration), and the pose is then refined by gradient
    descent on the signal loss (`fit_pose`).  A radar cloud of a compact
    object has tens of points, too few to fix a rotation: registration is
    translation-only unless rotate=True or the target cloud has >= 200
    points."""
    dev = torch.device(device)
    sim = Simulator(template, dev)
    tgt = sim.point_cloud(target_cube, pfa=pfa, snr_db=snr_db, seed=1)[:, :3]
    src = sim.point_cloud(sim.forward().clone(), pfa=pfa, snr_db=snr_db, seed=2)[:, :3]
    c0 = chamfer_points(src, tgt)
    R, t = register_rigid(src, tgt, rotate=(len(tgt) >= 200) if rotate is None else rotate)
    # the pose acts about the template's vertex centroid: x' = R (x - c) + c + trans
    base = torch.as_tensor(template.verts, dtype=torch.float64, device=dev)
    c = base.mean(0)
    omega0 = rotation_to_axis_angle(R)
    trans0 = R @ c + t - c
    init_pts = rigid_pose(base.float(), omega0.float(), trans0.float())
    isim = Simulator(dataclasses.replace(template, verts=init_pts.cpu().numpy()), dev)
    c1 = chamfer_points(isim.point_cloud(isim.forward().clone(), pfa=pfa, snr_db=snr_db, seed=2)[:, :3], tgt)
    res = fit_pose(template, target_cube, steps=steps, lr=lr, omega0=tuple(omega0.tolist()),
                   trans0=tuple(trans0.tolist()), objective=objective, device=device)
    fin = rigid_pose(base.float(), torch.as_tensor(res.omega, device=dev), torch.as_tensor(res.trans, device=dev))
    fsim = Simulator(dataclasses.replace(template, verts=fin.cpu().numpy()), dev)
    c2 = chamfer_points(fsim.point_cloud(fsim.forward().clone(), pfa=pfa, snr_db=snr_db, seed=2)[:, :3], tgt)
    return CloudFitResult(omega0.cpu().numpy(), trans0.cpu().numpy(), res, c0, c1, c2, int(len(tgt)))


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="mesh reconstruction from a simulated IF cube")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--rays", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--log-every", type=int, default=20)
    ap.add_argument("--objective", default="heatmap", choices=["heatmap", "if"])
    ap.add_argument("--attached", action="store_true",
                    help="reparameterised gradient (Eqs. 6-7, samples follow their first hit)")
    args = ap.parse_args(argv)
    start, target = S.recon_scenes(n_rays=args.rays)
    res = reconstruct(start, target, steps=args.steps, lr=args.lr, log_every=args.log_every, objective=args.objective,
                      attached=args.attached)
    print(json.dumps({"workload": "recon_geodesic22_to_superquadric", "objective": args.objective, "steps": args.steps,
                      "gradient": "attached" if args.attached else "fixed-directions",
                      "ms_per_step_median": float(np.median(res.step_ms[1:] if len(res.step_ms) > 1 else res.step_ms)),
                      "loss_first": res.losses[0], "loss_last": res.losses[-1],
                      "chamfer_start": res.chamfer_start, "chamfer_final": res.chamfer_final, "lambda": res.lam}))


if __name__ == "__main__":
    main()
