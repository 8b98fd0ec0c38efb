"""torch.autograd bindings of the simulator (paper Sec. 3.3, Eq. 13).

`SBRFunction` maps mesh vertex positions to the complex IF cube; its
backward runs libsbr's hand-written adjoint (Eqs. 11-12 per path, then the
geometry reverse sweep to the vertices).  `RadarCubeFunction` is the
signal-to-image map T of the spatial loss (Eq. 16) and its conjugate
transpose.  `IFLoss` is sum |S - target|^2 with its gradient from libsbr.
PyTorch only holds memory and records the graph; the arithmetic runs in HIP.
"""
from __future__ import annotations

import torch

from .sbr import Hits, Simulator


class SBRFunction(torch.autograd.Function):
    """verts [nv,3] float32 -> IF cube [V,C,S] complex64.

    Each call traces into fresh hit records kept by the graph, so several
    forwards may be in flight before their backwards run.  With refit=True
    the BVH of the previous build is refit to the new vertices (same faces).
    With attached=True the gradient is that of the reparameterised estimator
    (Eqs. 6-7, samples follow their first hit), which moves silhouettes.
    """

    @staticmethod
    def forward(ctx, verts: torch.Tensor, sim: Simulator, refit: bool = True, attached: bool = False):
        sim.set_verts(verts)
        sim.build(refit=refit)
        sim.hits = Hits.empty(sim.K, sim.R, sim.device)
        sim.trace()
        cube = torch.view_as_complex(sim.synth())
        ctx.sim = sim
        ctx.paths_token = sim.paths_token   # this synthesis's path records in the scratch
        ctx.attached = attached
        ctx.hits = sim.hits
        ctx.verts = sim.mesh.verts.clone()
        return cube

    @staticmethod
    def backward(ctx, grad_cube: torch.Tensor):
        sim = ctx.sim
        # the hit records and vertex positions of this forward
        cur_hits, cur_verts = sim.hits, sim.mesh.verts.clone()
        sim.hits = ctx.hits
        sim.mesh.verts.copy_(ctx.verts)
        try:
            # reuse the path records if nothing has replaced them since this forward
            reuse = sim.paths_token is not None and sim.paths_token == ctx.paths_token
            g = sim.backward(grad_cube.contiguous(), attached=ctx.attached, reuse_paths=reuse)
        finally:
            sim.hits = cur_hits
            sim.mesh.verts.copy_(cur_verts)
        return g, None, None, None


class RadarCubeFunction(torch.autograd.Function):
    """IF cube [V,C,S] -> radar cube [Na,C,S] (range, Doppler, angle DFTs)."""

    @staticmethod
    def forward(ctx, cube: torch.Tensor, sim: Simulator, window: int = 0):
        ctx.sim, ctx.window = sim, window
        return sim.radar_cube(cube, direction=0, window=window)

    @staticmethod
    def backward(ctx, grad_X: torch.Tensor):
        return ctx.sim.radar_cube(grad_X.contiguous(), direction=1, window=ctx.window), None, None


class IFLoss(torch.autograd.Function):
    """L = scale * sum |S - target|^2 (libsbr's loss entry)."""

    @staticmethod
    def forward(ctx, cube: torch.Tensor, target: torch.Tensor, sim: Simulator, scale: float = 1.0):
        grad, loss = sim.loss_grad(cube, target)
        ctx.save_for_backward(grad)
        ctx.scale = scale
        return loss[0] * scale

    @staticmethod
    def backward(ctx, gl: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return torch.view_as_complex(grad) * (gl * ctx.scale), None, None, None


class HeatmapLoss(torch.autograd.Function):
    """L = scale * mean (|X|^2 - H)^2 over the radar cube X = T(S): the MSE of
    the spatial multi-antenna loss (Eq. 16) on the image |T(S)|^2."""

    @staticmethod
    def forward(ctx, X: torch.Tensor, H: torch.Tensor, sim: Simulator, scale: float = 1.0):
        grad, loss = sim.loss_grad(X, H, mode=1)
        ctx.save_for_backward(grad)
        ctx.scale = scale
        return loss[0] * scale

    @staticmethod
    def backward(ctx, gl: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return torch.view_as_complex(grad) * (gl * ctx.scale), None, None, None


def simulate(verts: torch.Tensor, sim: Simulator, refit: bool = True, attached: bool = False) -> torch.Tensor:
    return SBRFunction.apply(verts, sim, refit, attached)


def skew(w: torch.Tensor) -> torch.Tensor:
    """[w]x, the cross-product matrix of a 3-vector."""
    z = torch.zeros((), dtype=w.dtype, device=w.device)
    return torch.stack([torch.stack([z, -w[2], w[1]]), torch.stack([w[2], z, -w[0]]),
                        torch.stack([-w[1], w[0], z])])


def box_pose(base: torch.Tensor, log_scale: torch.Tensor, omega: torch.Tensor, trans: torch.Tensor,
             center: torch.Tensor = None) -> torch.Tensor:
    """3D bounding-box parameterisation (Sec. 3.1 (i), the object's
    transformation matrix): verts = exp([omega]x) diag(exp(log_scale))
    (base - c) + c + trans about the vertex centroid c."""
    c = base.mean(dim=0) if center is None else center
    R = torch.linalg.matrix_exp(skew(omega))
    return ((base - c) * torch.exp(log_scale)) @ R.T + c + trans


def rigid_pose(base: torch.Tensor, omega: torch.Tensor, trans: torch.Tensor,
               center: torch.Tensor = None) -> torch.Tensor:
    """Object-transform parameterisation of the geometry (Sec. 3.1 (i)):
    verts = exp([omega]x) (base - c) + c + trans, c = the vertex centroid
    unless given.  The gradients with respect to omega (axis-angle) and trans
    follow from dL/dverts by the chain rule (torch autograd)."""
    c = base.mean(dim=0) if center is None else center
    R = torch.linalg.matrix_exp(skew(omega))
    return (base - c) @ R.T + c + trans
