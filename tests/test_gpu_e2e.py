"""End-to-end parity: GPU build + trace + synthesis (+ loss + backward), every
stage on the HIP path, against the FP64 oracle's own trace, paths and sums.

The comparison mask follows the hit-id tolerance: a record flagged on either
side (near an edge, a tie, grazing, near t_min) is dropped on both sides with
the later bounces of its ray, so both sums run over the same paths.  Ids of
every other record must agree bit for bit (checked first).
"""
import numpy as np
import pytest

from paper_2311_13182_amd import scenes as S

from _parity import compare_trace, fd_coords_local, log, rel_l2, union_flags

pytestmark = pytest.mark.gpu

IF_TOL = 1e-4
GRAD_TOL = 1e-2


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_13182_amd import _lib
    _lib.load()
    return torch


def _gpu_trace(torch, sc):
    from paper_2311_13182_amd.sbr import Simulator
    sim = Simulator(sc, "cuda", cube=True)
    sim.trace()
    torch.cuda.synchronize()
    h = sim.hits
    g = {"tri": h.tri.cpu().numpy(), "t": h.t.cpu().numpy().astype(np.float64), "flags": h.flags.cpu().numpy()}
    return sim, g


def _masked(torch, sim, g, o):
    """Both sides' flags OR-ed into the device hit flags; returns the mask."""
    U = union_flags(g["flags"], o["flags"])
    sim.hits.flags.copy_(torch.as_tensor(U, device="cuda"))
    return U


def test_end_to_end_forward_and_determinism(torch_cuda, orc):
    torch = torch_cuda
    sc = S.trihedral_plate()
    sim, g = _gpu_trace(torch, sc)
    c1 = torch.view_as_complex(sim.synth()).clone()
    c2 = torch.view_as_complex(sim.synth()).clone()
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(c1), torch.view_as_real(c2))
    o = orc.trace(sc)
    n_chk, n_fl = compare_trace(g, o)
    U = _masked(torch, sim, g, o)
    cube = torch.view_as_complex(sim.synth()).cpu().numpy().astype(np.complex128)
    ref = orc.synth(sc, orc.paths(sc, o["tri"], U))
    e = rel_l2(cube, ref)
    log(f"end-to-end trihedral+plate: {n_chk} records checked, {n_fl} flagged (either side), rel L2 {e:.3e}")
    assert e <= IF_TOL
    # range peaks of the plate (bin 15) and the trihedral (bin 10)
    X = sim.radar_cube(c1)
    prof = np.abs(X.cpu().numpy()[0, 0])
    for want in (10, 15):
        j = want - 1 + int(np.argmax(prof[want - 1:want + 2]))
        assert prof[j] >= prof[j - 1] and prof[j] >= prof[j + 1]


def test_end_to_end_icosphere_full_grid(torch_cuda, orc):
    """Icosphere of 20,480 triangles, 512 x 512 rays, K = 3, 3 TX x 4 RX, 64
    chirps x 256 samples, scene moving at 1 m/s: GPU build + trace +
    synthesis vs the oracle's brute-force trace and direct sum on 24 sampled
    antenna-chirp rows (every id checked, all paths summed)."""
    torch = torch_cuda
    sc = S.icosphere_scene()
    assert sc.nf == 20480 and sc.grid.nx == 512 and sc.grid.max_bounces == 3
    assert sc.radar.n_virtual == 12 and sc.chirp.n_chirps == 64 and np.linalg.norm(sc.radar.vel) == 1.0
    sim, g = _gpu_trace(torch, sc)
    log("icosphere 512^2: GPU trace done, oracle trace of 262144 rays x 20480 triangles ...")
    o = orc.trace(sc)
    n_chk, n_fl = compare_trace(g, o)
    U = _masked(torch, sim, g, o)
    cube = torch.view_as_complex(sim.synth()).cpu().numpy().astype(np.complex128)
    p = orc.paths(sc, o["tri"], U)
    assert sim.n_paths() == len(p["amp"]) > 150000
    V, C, Sn = cube.shape
    rows = np.random.default_rng(2).choice(V * C, size=24, replace=False)
    rows[:2] = [0, V * C - 1]
    ref = orc.synth(sc, p, rows=rows)
    e = rel_l2(cube.reshape(V * C, Sn)[rows], ref)
    log(f"end-to-end icosphere 512^2: {n_chk} records checked, {n_fl} flagged (either side), "
        f"{len(p['amp'])} paths, rel L2 {e:.3e} on {len(rows)} rows")
    assert e <= IF_TOL


def test_end_to_end_backward_icosphere(torch_cuda, orc):
    """Icosphere of 20,480 triangles at 128 x 128 rays, 12 antennas x 8 chirps:
    GPU trace + synthesis + loss gradient + backward (every stage on the HIP
    path) vs the oracle's central differences of L = |S - S_target|^2 on 32
    random coordinates of hit vertices and along 8 random directions."""
    torch = torch_cuda
    sc = S.icosphere_scene(n_rays=128, n_chirps=8)
    tgt, _, _ = orc.forward(S.jitter(sc, 2e-3, 12))
    sim, g = _gpu_trace(torch, sc)
    o = orc.trace(sc)
    compare_trace(g, o)
    U = _masked(torch, sim, g, o)
    cube = torch.view_as_complex(sim.synth())
    grad_if, _ = sim.loss_grad(cube, torch.as_tensor(tgt.astype(np.complex64), device="cuda"))
    gv = sim.backward(grad_if).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(21)
    hit_v = np.unique(sc.faces[np.unique(o["tri"][o["tri"] >= 0])].reshape(-1))
    coords = np.sort(rng.choice(hit_v, size=32, replace=False) * 3 + rng.integers(0, 3, size=32))
    fd = fd_coords_local(orc, sc, o["tri"], U, tgt, coords)
    e_c = rel_l2(gv.reshape(-1)[coords], fd)
    errs = []
    for i in range(8):
        w = np.zeros((sc.nv, 3))
        w[hit_v] = rng.normal(size=(len(hit_v), 3))
        w /= np.linalg.norm(w)
        fdw = orc.fd_directional(sc, o["tri"], U, tgt, w, h=1e-9)
        errs.append(abs(float((gv * w).sum()) - fdw) / abs(fdw))
    log(f"end-to-end backward icosphere 128^2 C=8: 32 coordinates rel L2 {e_c:.3e}; "
        f"8 directions max rel {max(errs):.3e}")
    assert e_c <= GRAD_TOL and max(errs) <= GRAD_TOL
