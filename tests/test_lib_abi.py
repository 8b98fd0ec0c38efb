"""The C-ABI library loads, exports every symbol include/sbr.h declares, and
rejects bad arguments before enqueueing anything.  CPU only: no call here
reaches a GPU kernel."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sbr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sbr_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2311_13182_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2311_13182_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    from paper_2311_13182_amd import _lib as L
    decl = _declared()
    assert len(decl) == 21
    assert sorted(L.EXPORTS) == decl
    for name in decl:
        assert hasattr(lib, name), name


def test_size_queries(lib):
    from paper_2311_13182_amd import _lib as L
    from paper_2311_13182_amd import scenes as S
    from paper_2311_13182_amd import sbr
    assert lib.sbr_bvh_bytes(0) == 0
    b1, b2 = lib.sbr_bvh_bytes(1), lib.sbr_bvh_bytes(1000)
    assert 0 < b1 < b2
    sc = S.icosphere_scene(level=1, n_rays=16, n_chirps=4)
    r, g, c = sbr.radar_struct(sc.radar), sbr.rays_struct(sc.grid), sbr.chirp_struct(sc.chirp)
    syn = lib.sbr_scratch_bytes(L.SBR_OP_SYNTH, None, ct.byref(g), ct.byref(r), ct.byref(c))
    bwd = lib.sbr_scratch_bytes(L.SBR_OP_BACKWARD, None, ct.byref(g), ct.byref(r), ct.byref(c))
    assert syn > 0 and bwd > 0
    # paths scale with rays x bounces
    g2 = sbr.rays_struct(sc.grid.__class__(32, 32, 0.1, 0.1, 3))
    assert lib.sbr_scratch_bytes(L.SBR_OP_SYNTH, None, ct.byref(g2), ct.byref(r), ct.byref(c)) > syn
    assert lib.sbr_scratch_bytes(99, None, None, None, None) == 0
    assert lib.sbr_scratch_bytes(L.SBR_OP_SYNTH, None, None, None, None) == 0


def _gpu_visible() -> bool:
    import torch
    return torch.cuda.device_count() > 0


@pytest.mark.skipif(_gpu_visible(), reason="passes made-up device addresses; runs only where no GPU is visible, "
                                           "so no kernel can ever receive them")
def test_argument_errors_are_reported(lib):
    from paper_2311_13182_amd import _lib as L
    from paper_2311_13182_amd import scenes as S
    from paper_2311_13182_amd import sbr
    fake = ct.c_void_p(0x10000)   # never dereferenced: checks fail first
    assert lib.sbr_trace(None, None, None, None, None, None, None) == L.SBR_E_ARG
    assert b"mesh" in lib.sbr_last_error()
    sc = S.icosphere_scene(level=1, n_rays=16, n_chirps=4)
    m = L.sbr_mesh(0x10000, sc.nv, 0x20000, sc.nf, None)
    r, g, c = sbr.radar_struct(sc.radar), sbr.rays_struct(sc.grid), sbr.chirp_struct(sc.chirp)
    h = L.sbr_hits(0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    bad = sbr.rays_struct(sc.grid.__class__(16, 16, 0.1, 0.1, 9))
    assert lib.sbr_trace(ct.byref(m), fake, ct.byref(r), ct.byref(bad), ct.byref(h), None, None) == L.SBR_E_ARG
    assert b"max_bounces" in lib.sbr_last_error()
    # scratch too small -> SBR_E_SCRATCH with the required size in the message
    rc = lib.sbr_synth_if(ct.byref(m), None, 0, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c), 1, fake,
                          fake, 16, None)
    assert rc == L.SBR_E_SCRATCH and b"needed" in lib.sbr_last_error()
    rc = lib.sbr_backward(ct.byref(m), None, 0, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c), 1, fake,
                          fake, None, fake, 16, None)
    assert rc == L.SBR_E_SCRATCH
    # SBR_PATHS_IN_SCRATCH belongs to sbr_backward only
    rc = lib.sbr_synth_if(ct.byref(m), None, 0, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c),
                          1 | L.SBR_PATHS_IN_SCRATCH, fake, fake, 1 << 40, None)
    assert rc == L.SBR_E_ARG and b"unknown flags" in lib.sbr_last_error()
    rc = lib.sbr_backward(ct.byref(m), None, 0, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c),
                          1 | L.SBR_PATHS_IN_SCRATCH, fake, fake, None, fake, 16, None)
    assert rc == L.SBR_E_SCRATCH
    pg = L.sbr_param_grads(0x10000, None)     # material gradients need a material table
    rc = lib.sbr_backward(ct.byref(m), None, 0, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c), 1, fake,
                          fake, ct.byref(pg), fake, 1 << 30, None)
    assert rc == L.SBR_E_ARG and b"material" in lib.sbr_last_error()
    # radar cube: n_angle below V, bad window, bad direction
    assert lib.sbr_radar_cube(fake, 12, 8, 16, 8, 0, 0, fake, fake, 1 << 30, None) == L.SBR_E_ARG
    assert lib.sbr_radar_cube(fake, 12, 8, 16, 64, 2, 0, fake, fake, 1 << 30, None) == L.SBR_E_ARG
    assert lib.sbr_radar_cube(fake, 12, 8, 16, 64, 0, 5, fake, fake, 1 << 30, None) == L.SBR_E_ARG
    # planar cube: angle grid smaller than the array, size query
    assert lib.sbr_radar_cube_2d(fake, 20, 20, 8, 16, 16, 64, 0, 0, fake, fake, 1 << 30, None) == L.SBR_E_ARG
    assert lib.sbr_radar_cube_2d_bytes(20, 20, 8, 16, 8, 64) == 0
    assert lib.sbr_radar_cube_2d_bytes(20, 20, 8, 16, 64, 64) >= 2 * 8 * 20 * 64 * 8 * 16
    # too many antennas
    rr = sbr.radar_struct(sc.radar)
    rr.n_tx, rr.n_rx = L.SBR_MAX_TX + 1, 4
    assert lib.sbr_synth_if(ct.byref(m), None, 0, ct.byref(rr), ct.byref(g), ct.byref(h), ct.byref(c), 1, fake,
                            fake, 1 << 40, None) == L.SBR_E_ARG
    # material modes outside {0,1,2}
    mats = (L.sbr_material * 1)()
    mats[0].mode = 7
    assert lib.sbr_synth_if(ct.byref(m), mats, 1, ct.byref(r), ct.byref(g), ct.byref(h), ct.byref(c), 1, fake,
                            fake, 1 << 40, None) == L.SBR_E_ARG
    # CFAR: bad pfa
    assert lib.sbr_cfar(fake, 4, 8, 16, 2, 8, ct.c_double(2.0), fake, None, 10, fake, fake, 1 << 30,
                        None) == L.SBR_E_ARG
    # CFAR: sizes beyond the documented limits
    assert lib.sbr_cfar(fake, 4, 8192, 16, 2, 8, ct.c_double(1e-4), fake, None, 10, fake, fake, 1 << 30,
                        None) == L.SBR_E_ARG
    # BVH: empty mesh
    m0 = L.sbr_mesh(None, 0, None, 0, None)
    assert lib.sbr_build_bvh(ct.byref(m0), fake, 1 << 20, 0, fake, 1 << 20, None) == L.SBR_E_ARG
    # batched calls: table size query, table too small, a bad request named
    assert lib.sbr_batch_table_bytes(0) == 0 and lib.sbr_batch_table_bytes(L.SBR_MAX_BATCH + 1) == 0
    assert 0 < lib.sbr_batch_table_bytes(1) < lib.sbr_batch_table_bytes(64)
    reqs = (L.sbr_request * 2)()
    for q in reqs:
        q.mesh, q.radar, q.rays, q.hits, q.chirp = ct.pointer(m), ct.pointer(r), ct.pointer(g), ct.pointer(h), \
            ct.pointer(c)
        q.flags, q.if_cube, q.grad_if, q.grad_verts, q.scratch, q.scratch_bytes = 1, fake, fake, fake, fake, 1 << 40
    assert lib.sbr_synth_if_batched(reqs, 2, fake, 16, None) == L.SBR_E_SCRATCH
    reqs[1].scratch_bytes = 16
    rc = lib.sbr_synth_if_batched(reqs, 2, fake, 1 << 20, None)
    assert rc == L.SBR_E_SCRATCH and lib.sbr_last_error().startswith(b"request 1:")
    reqs[1].scratch_bytes = 1 << 40
    reqs[0].rays = ct.pointer(bad)
    rc = lib.sbr_backward_batched(reqs, 2, fake, 1 << 20, None)
    assert rc == L.SBR_E_ARG and b"request 0" in lib.sbr_last_error() and b"max_bounces" in lib.sbr_last_error()
    assert lib.sbr_synth_if_batched(reqs, -1, fake, 1 << 20, None) == L.SBR_E_ARG
    assert lib.sbr_backward_batched(reqs, L.SBR_MAX_BATCH + 1, fake, 1 << 30, None) == L.SBR_E_ARG
    # two valid requests that write the same device bytes are refused before anything is enqueued
    reqs[0].rays = ct.pointer(g)
    for fn in (lib.sbr_synth_if_batched, lib.sbr_backward_batched):
        rc = fn(reqs, 2, fake, 1 << 20, None)
        assert rc == L.SBR_E_ARG and b"share device memory" in lib.sbr_last_error(), lib.sbr_last_error()


def test_product_path_fails_loudly_without_library(tmp_path):
    from paper_2311_13182_amd import _lib as L
    with pytest.raises(ImportError):
        L._lib_backup = L._lib
        try:
            L._lib = None
            L.load(str(tmp_path / "missing.so"))
        finally:
            L._lib = L._lib_backup


def test_binding_checks_buffers_before_the_call():
    """The binding refuses buffers the C ABI would overrun or misread (it
    cannot see their sizes): wrong dtype, too few elements, non-contiguous,
    host memory."""
    import torch
    from paper_2311_13182_amd import sbr
    f32 = torch.zeros(8, dtype=torch.float32)
    with pytest.raises(ValueError, match="float32"):
        sbr._buf(torch.zeros(8, dtype=torch.float64), torch.float32, 8, "x")
    with pytest.raises(ValueError, match="needed"):
        sbr._buf(f32, torch.float32, 9, "x")
    with pytest.raises(ValueError, match="contiguous"):
        sbr._buf(torch.zeros(4, 4)[:, 1], torch.float32, 4, "x")
    with pytest.raises(ValueError, match="device memory"):
        sbr._buf(f32, torch.float32, 8, "x")
    assert sbr._buf(None, torch.float32, 8, "x", optional=True) is None
    with pytest.raises(ValueError, match="required"):
        sbr._buf(None, torch.float32, 8, "x")
    # an IF cube one sample short is refused before anything reaches the library
    from paper_2311_13182_amd import scenes as S
    sc = S.trihedral_plate()
    h = sbr.Hits.empty(sc.grid.max_bounces, sc.grid.n_rays, "cpu")
    short = torch.zeros(2 * sc.radar.n_virtual * sc.chirp.n_chirps * sc.chirp.n_samples - 1)
    with pytest.raises(ValueError, match="if_cube"):
        sbr.sbr_synth_if(None, sc.radar, sc.grid, h, sc.chirp, 0, short, torch.zeros(16, dtype=torch.uint8))
