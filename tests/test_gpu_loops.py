"""GPU tests of the layers above the kernels: BVH refit, the autograd
Function, the reconstruction loop (with checkpoint/resume) and the serving
loop (each result alone == in the mix; requests overlap on the device)."""
import dataclasses
import math
import os

import numpy as np
import pytest

from paper_2311_13182_amd import scenes as S

from _parity import device_hits_from_oracle, log, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_13182_amd import _lib
    _lib.load()
    return torch


def test_refit_matches_rebuild(torch_cuda):
    torch = torch_cuda
    from paper_2311_13182_amd.sbr import Simulator
    sc = S.icosphere_scene(level=4, n_rays=96, n_chirps=1)
    a = Simulator(sc, "cuda")
    a.build()
    moved = S.jitter(sc, 5e-4, 21)
    a.set_verts(torch.as_tensor(moved.verts, device="cuda"))
    a.build(refit=True)
    a.trace()
    b = Simulator(moved, "cuda")
    b.build()
    b.trace()
    torch.cuda.synchronize()
    for f in ("tri", "t", "u", "v", "flags"):
        assert torch.equal(getattr(a.hits, f), getattr(b.hits, f)), f


def test_autograd_gradient_matches_oracle(torch_cuda, orc):
    torch = torch_cuda
    from paper_2311_13182_amd.autograd import IFLoss, SBRFunction
    from paper_2311_13182_amd.sbr import Simulator
    sc = S.icosphere_scene(level=3, n_rays=48, n_chirps=4)
    tsc = S.jitter(sc, 1e-3, 31)
    tgt_np, _, _ = orc.forward(tsc)
    sim = Simulator(sc, "cuda")
    verts = torch.as_tensor(sc.verts, device="cuda").requires_grad_(True)
    tgt = torch.as_tensor(tgt_np.astype(np.complex64), device="cuda")
    loss = IFLoss.apply(SBRFunction.apply(verts, sim, False), tgt, sim, 1.0)
    loss.backward()
    g = verts.grad.detach().cpu().numpy().astype(np.float64)
    o = orc.trace(sc)
    rng = np.random.default_rng(8)
    errs = []
    for _ in range(3):
        w = rng.normal(size=g.shape)
        w /= np.linalg.norm(w)
        fd = orc.fd_directional(sc, o["tri"], o["flags"], tgt_np, w, h=1e-9)
        errs.append(abs(float((g * w).sum()) - fd) / abs(fd))
    log(f"autograd vs oracle FD rel errs {errs}")
    assert max(errs) <= 1e-2


def test_radar_cube_function_adjoint(torch_cuda):
    torch = torch_cuda
    from paper_2311_13182_amd.autograd import RadarCubeFunction
    from paper_2311_13182_amd.sbr import Simulator
    sc = S.icosphere_scene(level=1, n_rays=8, n_chirps=8).with_chirp(n_samples=32)
    sim = Simulator(sc, "cuda")
    x = torch.randn(12, 8, 32, dtype=torch.complex64, device="cuda", requires_grad=True)
    X = RadarCubeFunction.apply(x, sim, 1)
    H = torch.rand(64, 8, 32, device="cuda")
    loss = ((X.abs() ** 2 - H) ** 2).mean()
    loss.backward()
    # reference: the same loss through torch.fft on the CPU in float64
    xc = x.detach().cpu().to(torch.complex128).requires_grad_(True)
    w = torch.as_tensor(np.hanning(32)) [None, None, :] * torch.as_tensor(np.hanning(8))[None, :, None]
    Xr = torch.fft.fft(torch.fft.fft(torch.fft.fft(xc * w, dim=2), dim=1), n=64, dim=0)
    lr = ((Xr.abs() ** 2 - H.cpu().double()) ** 2).mean()
    lr.backward()
    assert rel_l2(x.grad.cpu().numpy(), xc.grad.numpy()) <= 1e-4


def test_recon_loop_decreases_and_resumes(torch_cuda, tmp_path):
    from paper_2311_13182_amd import recon
    start, target = S.recon_scenes(n_rays=96, n_chirps=8)
    ck = str(tmp_path / "ck.pt")
    # 0.1 mm steps: the phase of a path turns by 2 pi per 1.95 mm of range
    res = recon.reconstruct(start, target, steps=40, lr=1e-4, checkpoint=ck)
    log(f"recon: loss {res.losses[0]:.4f} -> {res.losses[-1]:.4f}, chamfer {res.chamfer_start:.3e} -> "
        f"{res.chamfer_final:.3e}, ms/step {np.median(res.step_ms):.1f}")
    assert res.losses[-1] < 0.1 * res.losses[0]
    # resume from the step-20 checkpoint written during a 20-step run
    ck2 = str(tmp_path / "ck2.pt")
    recon.reconstruct(start, target, steps=20, lr=1e-4, checkpoint=ck2)
    res2 = recon.reconstruct(start, target, steps=40, lr=1e-4, resume=ck2)
    assert rel_l2(res2.verts, res.verts) <= 1e-4


def _serving_requests():
    reqs = S.serving_requests(n=10, qps=1.0, seed=77, grids=(64, 96, 128), nf_range=(500, 5000), chirps=(8, 16))
    return reqs


def test_serving_alone_equals_mix_and_overlaps(torch_cuda, orc):
    torch = torch_cuda
    from paper_2311_13182_amd.serve import GPUExecutor, Request, Scheduler, run_sequential
    reqs = _serving_requests()
    ex = GPUExecutor(n_streams=4)
    for r in reqs:
        if r.backward:
            h = ex.launch(Request(-1, S.jitter(r.scene, 2e-3, 33 + r.rid)))
            r.target = ex.collect(h)["cube"]
            ex.release(h)
    plain = [Request(r.rid, r.scene, r.backward, r.target, 0.0) for r in reqs]
    alone = run_sequential(ex, plain)
    sch = Scheduler(ex, budget_bytes=8 << 30, max_active=8)
    sch.start()
    futs = [sch.submit(Request(r.rid, r.scene, r.backward, r.target, 0.0)) for r in reqs]
    mix = [f.result(timeout=300) for f in futs]
    sch.stop()
    assert all(m.status == "ok" for m in mix), [m.error for m in mix]
    for a, m in zip(alone, mix):
        assert a.n_paths == m.n_paths > 0
        assert np.array_equal(a.cube.view(np.uint32), m.cube.view(np.uint32)), a.rid
        if a.grad is not None:
            assert rel_l2(m.grad, a.grad) <= 1e-5
    # in flight together: some request was admitted before another finished
    iv = sorted((m.t_admit, m.t_done) for m in mix)
    assert any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))
    # a served result equals a fresh single-request simulation of the same scene
    from paper_2311_13182_amd.sbr import Simulator
    fresh = Simulator(reqs[0].scene, "cuda").forward().cpu().numpy()
    assert np.array_equal(fresh.view(np.uint32), mix[0].cube.view(np.uint32))


def test_rigid_pose_gradient_matches_oracle(torch_cuda, orc):
    """Object-transform parameters (axis-angle + translation) through
    SBRFunction's vertex gradient vs central differences of the oracle with the
    same transform applied in FP64."""
    torch = torch_cuda
    from paper_2311_13182_amd.autograd import IFLoss, SBRFunction, rigid_pose
    from paper_2311_13182_amd.sbr import Simulator
    sc = S.icosphere_scene(level=3, n_rays=48, n_chirps=4)
    tgt_np, _, _ = orc.forward(S.jitter(sc, 1e-3, 32))
    sim = Simulator(sc, "cuda")
    base = torch.as_tensor(sc.verts, device="cuda")
    omega = torch.zeros(3, device="cuda", requires_grad=True)
    trans = torch.zeros(3, device="cuda", requires_grad=True)
    tgt = torch.as_tensor(tgt_np.astype(np.complex64), device="cuda")
    loss = IFLoss.apply(SBRFunction.apply(rigid_pose(base, omega, trans), sim, False), tgt, sim, 1.0)
    loss.backward()
    an = np.concatenate([omega.grad.cpu().numpy(), trans.grad.cpu().numpy()]).astype(np.float64)
    o = orc.trace(sc)
    b64 = sc.verts.astype(np.float64)
    c = b64.mean(axis=0)

    def pose(k):
        def f(s, d):
            if k < 3:
                K = np.zeros((3, 3))
                i, j = (k + 1) % 3, (k + 2) % 3
                K[i, j], K[j, i] = -1.0, 1.0          # [e_k]x
                R = np.eye(3) + math.sin(d) * K + (1.0 - math.cos(d)) * (K @ K)
                v = (b64 - c) @ R.T + c
            else:
                v = b64 + d * np.eye(3)[k - 3]
            return dataclasses.replace(s, verts=v)
        return f

    fd = np.array([orc.fd_scene(sc, o["tri"], o["flags"], tgt_np, pose(k), 1e-8 if k < 3 else 1e-9)
                   for k in range(6)])
    log(f"rigid pose gradient gpu {an} fd {fd}")
    assert rel_l2(an[:3], fd[:3]) <= 1e-2
    assert rel_l2(an[3:], fd[3:]) <= 1e-2


def test_fit_pose_converges_locally(torch_cuda):
    """Pose fit on the IF loss from a start within a quarter wavelength of the
    true pose recovers it (the loss is phase-periodic in range, so this is a
    local test)."""
    torch = torch_cuda
    from paper_2311_13182_amd.autograd import rigid_pose
    from paper_2311_13182_amd.recon import fit_pose
    from paper_2311_13182_amd.sbr import Simulator
    _, sc = S.recon_scenes(n_rays=96, n_chirps=8)
    w_true = np.array([0.0, 0.05, 0.03])
    t_true = np.array([0.01, -0.008, 0.02])
    base = torch.as_tensor(sc.verts, device="cuda")
    posed = rigid_pose(base, torch.tensor(w_true, dtype=torch.float32, device="cuda"),
                       torch.tensor(t_true, dtype=torch.float32, device="cuda"))
    tcube = Simulator(dataclasses.replace(sc, verts=posed.cpu().numpy()), "cuda").forward().clone()
    w0 = w_true + np.array([1e-3, -1e-3, 5e-4])
    t0 = t_true + np.array([2e-4, -2e-4, 3e-4])
    r = fit_pose(sc, tcube, steps=120, lr=3e-5, omega0=w0, trans0=t0, objective="if")
    ew0, et0 = np.linalg.norm(w0 - w_true), np.linalg.norm(t0 - t_true)
    ew, et = np.linalg.norm(r.omega - w_true), np.linalg.norm(r.trans - t_true)
    log(f"fit_pose: loss {r.losses[0]:.3e} -> {r.losses[-1]:.3e}; |dw| {ew0:.2e} -> {ew:.2e} rad, "
        f"|dt| {et0:.2e} -> {et:.2e} m; {np.median(r.step_ms):.1f} ms/step")
    assert r.losses[-1] < 0.05 * r.losses[0]
    assert ew < 0.2 * ew0 and et < 0.2 * et0


def test_cloud_entry_vs_oracle(torch_cuda, orc):
    """sbr_cloud (detections -> world points) against the oracle's formulas,
    linear and planar arrays, a rotated and shifted radar."""
    torch = torch_cuda
    from paper_2311_13182_amd.sbr import Simulator
    rng = np.random.default_rng(12)
    for planar in (False, True):
        sc = S.imaging_scene(n_rays=16, n_chirps=16, n_samples=128) if planar else \
            S.icosphere_scene(level=1, n_rays=16, n_chirps=16).with_chirp(n_samples=128)
        c, s_ = math.cos(0.3), math.sin(0.3)
        rd = dataclasses.replace(sc.radar, origin=np.array([0.2, -0.1, 0.05]),
                                 rot=np.array([[c, 0.0, s_], [0.0, 1.0, 0.0], [-s_, 0.0, c]]))
        sc = dataclasses.replace(sc, radar=rd)
        sim = Simulator(sc, "cuda")
        n_ax, n_ay = (sim.n_ax, sim.n_ay) if planar else (sim.n_angle, 1)
        pts = np.stack([rng.integers(0, 128, 300), rng.integers(0, 16, 300), rng.integers(0, n_ax * n_ay, 300),
                        np.zeros(300, int)], 1).astype(np.int32)
        got = sim.cloud(torch.as_tensor(pts, device="cuda"),
                        torch.tensor([250], dtype=torch.int32, device="cuda")).cpu().numpy()
        want = orc.cloud(sc, pts[:250], n_ax, n_ay)
        assert np.isnan(got[250:]).all()
        assert np.allclose(got[:250], want, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("n_ax,n_ay", [(64, 1), (32, 24)])
def test_angle_peaks_vs_oracle(torch_cuda, orc, n_ax, n_ay):
    torch = torch_cuda
    from paper_2311_13182_amd.sbr import sbr_angle_peaks
    rng = np.random.default_rng(13)
    C, Sn = 8, 48
    X = (rng.normal(size=(n_ax * n_ay, C, Sn)) + 1j * rng.normal(size=(n_ax * n_ay, C, Sn))).astype(np.complex64)
    det = np.array([[r, d, 0, 0] for d in range(C) for r in range(1, Sn, 5)], np.int32)
    for rel in (0.0, 0.25):
        pts, n = sbr_angle_peaks(torch.as_tensor(X, device="cuda"), n_ax, n_ay, C, Sn,
                                 torch.as_tensor(det, device="cuda"),
                                 torch.tensor([len(det)], dtype=torch.int32, device="cuda"), rel=rel)
        n = int(n.item())
        want = orc.angle_peaks(X.astype(np.complex128), n_ax, n_ay, det, rel)
        log(f"angle peaks {n_ax}x{n_ay} rel {rel}: gpu {n} oracle {len(want)}")
        assert n == len(want) and np.array_equal(pts[:n].cpu().numpy(), want)


def test_fit_from_point_cloud(torch_cuda):
    """Fig. 1 from a measurement: the target's point cloud initialises the pose
    by registration, the signal loss refines it."""
    torch = torch_cuda
    from paper_2311_13182_amd.autograd import rigid_pose
    from paper_2311_13182_amd.recon import fit_from_point_cloud
    from paper_2311_13182_amd.sbr import Simulator
    obj, fo = S.superquadric_object(7, 100, 51, (0.2, 0.12, 0.15), (0.0, 0.0, 1.5))
    sc = S.Scene("template", obj.astype(np.float32), fo.astype(np.int32), S.planar_radar(20, 20, 62e9),
                 S.Chirp(fc=62e9, slope=7e9 / 25.6e-6, fs=10e6, n_samples=256, n_chirps=16),
                 S.Grid(192, 192, 0.3, 0.3, 2))
    w_true = np.array([0.0, 0.12, 0.05])
    t_true = np.array([0.06, -0.04, 0.1])
    posed = rigid_pose(torch.as_tensor(sc.verts, device="cuda"), torch.tensor(w_true, dtype=torch.float32,
                       device="cuda"), torch.tensor(t_true, dtype=torch.float32, device="cuda"))
    tcube = Simulator(dataclasses.replace(sc, verts=posed.cpu().numpy()), "cuda").forward().clone()
    r = fit_from_point_cloud(sc, tcube, steps=60, lr=2e-3)
    e0 = np.linalg.norm(t_true)
    e1 = np.linalg.norm(r.trans_init - t_true)
    e2 = np.linalg.norm(r.pose.trans - t_true)
    log(f"point-cloud fit: {r.n_target_points} target points; cloud Chamfer {r.chamfer_cloud_start:.3e} -> "
        f"{r.chamfer_cloud_init:.3e} (registered) -> {r.chamfer_cloud_final:.3e} (signal fit); |dt| {e0:.3f} -> "
        f"{e1:.3f} -> {e2:.3f} m; |dw| {np.linalg.norm(w_true):.3f} -> {np.linalg.norm(r.omega_init - w_true):.3f} "
        f"-> {np.linalg.norm(r.pose.omega - w_true):.3f}; loss {r.pose.losses[0]:.3e} -> {r.pose.losses[-1]:.3e}")
    assert r.n_target_points >= 10
    assert r.chamfer_cloud_init < 0.7 * r.chamfer_cloud_start
    assert e1 < 0.35 * e0
    assert min(r.pose.losses) < r.pose.losses[0]


def test_box_pose_gradient_matches_oracle(torch_cuda, orc):
    """3D bounding-box parameters (log scales) through SBRFunction's vertex
    gradient vs central differences of the oracle with the same anisotropic
    scaling applied in FP64."""
    torch = torch_cuda
    from paper_2311_13182_amd.autograd import IFLoss, SBRFunction, box_pose
    from paper_2311_13182_amd.sbr import Simulator
    sc = S.icosphere_scene(level=3, n_rays=48, n_chirps=4)
    tgt_np, _, _ = orc.forward(S.jitter(sc, 1e-3, 35))
    sim = Simulator(sc, "cuda")
    base = torch.as_tensor(sc.verts, device="cuda")
    ls = torch.zeros(3, device="cuda", requires_grad=True)
    z = torch.zeros(3, device="cuda")
    loss = IFLoss.apply(SBRFunction.apply(box_pose(base, ls, z, z), sim, False), torch.as_tensor(
        tgt_np.astype(np.complex64), device="cuda"), sim, 1.0)
    loss.backward()
    an = ls.grad.cpu().numpy().astype(np.float64)
    o = orc.trace(sc)
    b64 = sc.verts.astype(np.float64)
    c = b64.mean(axis=0)

    def scale(k):
        return lambda s, d: dataclasses.replace(s, verts=(b64 - c) * np.exp(d * np.eye(3)[k]) + c)

    fd = np.array([orc.fd_scene(sc, o["tri"], o["flags"], tgt_np, scale(k), 1e-8) for k in range(3)])
    log(f"box pose (log-scale) gradient gpu {an} fd {fd}")
    assert rel_l2(an, fd) <= 1e-2


def test_plain_c_abi_caller(torch_cuda, orc, tmp_path):
    """The C ABI used from C++ with hipMalloc and no Python: build, trace,
    synthesis and the radar cube of the trihedral + plate scene equal the
    Python binding's results bit for bit, and the oracle's IF cube to 1e-4."""
    import subprocess
    from paper_2311_13182_amd import _lib as L
    from paper_2311_13182_amd.sbr import Simulator, chirp_struct, radar_struct, rays_struct
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "sbr_c_example")
    assert os.path.exists(exe), "tests/c_abi/sbr_c_example is not built (run __graft_entry__.build())"
    sc = S.trihedral_plate()
    f = tmp_path / "scene.bin"
    with open(f, "wb") as fh:
        fh.write(np.array([sc.nv, sc.nf], np.int32).tobytes())
        fh.write(np.ascontiguousarray(sc.verts, np.float32).tobytes())
        fh.write(np.ascontiguousarray(sc.faces, np.int32).tobytes())
        for st in (radar_struct(sc.radar), rays_struct(sc.grid), chirp_struct(sc.chirp)):
            fh.write(bytes(st))
    out = tmp_path / "out.bin"
    log(f"running {exe}")
    r = subprocess.run([exe, str(f), str(out)], capture_output=True, text=True, timeout=120)
    log(f"  rc {r.returncode}: {r.stdout.strip()} {r.stderr.strip()[-300:]}")
    assert r.returncode == 0
    V, C, Sn = sc.radar.n_virtual, sc.chirp.n_chirps, sc.chirp.n_samples
    raw = np.fromfile(out, np.float32)
    cube_c = raw[:V * C * Sn * 2].reshape(V, C, Sn, 2)
    img_c = raw[V * C * Sn * 2:].reshape(64, C, Sn, 2)
    sim = Simulator(sc, "cuda")
    cube = sim.forward()
    img = torch_cuda.view_as_real(sim.radar_cube(cube))
    assert np.array_equal(cube_c, torch_cuda.view_as_real(cube).cpu().numpy())
    assert np.array_equal(img_c, img.cpu().numpy())
    ref, _, _ = orc.forward(sc)
    assert rel_l2(cube_c[..., 0] + 1j * cube_c[..., 1], ref) <= 1e-4


def test_step_captured_in_a_hip_graph(torch_cuda):
    """The library only enqueues kernels (no allocation, no memset, no host
    synchronisation), so one forward + backward step -- trace, synthesis,
    radar cube, IF-loss gradient, synthesis and geometry adjoints -- can be
    captured in a HIP graph and replayed.  Each of three replays, with eager
    work and synchronisations between them, matches the eager step: cube and
    image bit for bit, vertex gradient to 1e-6 (floating-point atomics)."""
    torch = torch_cuda
    from paper_2311_13182_amd.sbr import Simulator
    sc = S.icosphere_scene(level=3, n_rays=96, n_chirps=8)
    tsc = S.jitter(sc, 1e-3, 37)
    ref = Simulator(tsc, "cuda")
    target = ref.forward().clone()
    sim = Simulator(sc, "cuda")
    sim.build()
    cube = torch.empty((sim.V, sim.C, sim.S, 2), dtype=torch.float32, device="cuda")
    grad = torch.empty_like(cube)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    gv = torch.zeros((sim.mesh.nv, 3), dtype=torch.float32, device="cuda")
    tgt = torch.view_as_real(target).contiguous()

    def step():
        sim.trace()
        sim.synth(cube)
        img = sim.radar_cube(cube)
        sim.loss_grad(cube, tgt, grad, loss)
        gv.zero_()
        sim.backward(grad, grad_verts=gv)
        return img

    img_e = step()
    torch.cuda.synchronize()
    want = (cube.clone(), img_e.clone(), gv.clone(), loss.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                       # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        img_g = step()
    for rep in range(3):
        cube.zero_()
        gv.fill_(1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(cube, want[0]), rep
        assert torch.equal(img_g, want[1]), rep
        assert torch.equal(loss, want[3]), rep
        e = float((gv - want[2]).norm() / want[2].norm())
        log(f"graph replay {rep}: cube and image bit-exact, loss {float(loss):.6e}, gradient rel {e:.2e}")
        assert e <= 1e-6
        sim.trace()                  # eager work between replays
        torch.cuda.synchronize()
