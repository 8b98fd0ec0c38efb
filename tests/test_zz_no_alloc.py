"""The scratch-free radar cube entry point (sbr_radar_cube_noalloc, for
callers that cannot allocate) against sbr_radar_cube with a caller scratch:
two calls in a row through the C ABI, the second smaller, both directions."""
import ctypes as ct

import numpy as np
import pytest

from _parity import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_13182_amd import _lib
    _lib.load()
    return torch


def _both(torch, x, V, C, Sn, Na, window, direction):
    from paper_2311_13182_amd import _lib as L
    lib = L.load()
    shape_out = (Na, C, Sn, 2) if direction == 0 else (V, C, Sn, 2)
    a = torch.full(shape_out, float("nan"), device="cuda")
    b = torch.full(shape_out, float("nan"), device="cuda")
    st = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    need = max(1, int(lib.sbr_radar_cube_2d_bytes(V, 1, C, Sn, Na, 1)))
    scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
    L.check(lib.sbr_radar_cube(ct.c_void_p(x.data_ptr()), V, C, Sn, Na, window, direction, ct.c_void_p(a.data_ptr()),
                               ct.c_void_p(scratch.data_ptr()), need, st))
    del scratch
    base = torch.cuda.memory_allocated()
    L.check(lib.sbr_radar_cube_noalloc(ct.c_void_p(x.data_ptr()), V, C, Sn, Na, window, direction,
                                       ct.c_void_p(b.data_ptr()), st))
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    return a, b


def test_noalloc_cube_equals_scratch_entry_point(torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(17)
    cases = [((12, 128, 256), 64, 0), ((5, 7, 40), 64, 1)]   # full benchmark cube, then a smaller one
    for (V, C, Sn), Na, window in cases:
        for direction in (0, 1):
            shape = (V, C, Sn) if direction == 0 else (Na, C, Sn)
            x = torch.as_tensor((rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64),
                                device="cuda")
            xf = torch.view_as_real(x).contiguous()
            a, b = _both(torch, xf, V, C, Sn, Na, window, direction)
            assert torch.isfinite(a).all()
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (V, C, Sn, window, direction)
            log(f"no-alloc cube {V}x{C}x{Sn} -> {Na} window {window} direction {direction}: bit-exact")


def test_noalloc_cube_refuses_sizes_beyond_its_array(torch_cuda):
    torch = torch_cuda
    from paper_2311_13182_amd import _lib as L
    lib = L.load()
    x = torch.zeros(16, device="cuda")
    rc = lib.sbr_radar_cube_noalloc(ct.c_void_p(x.data_ptr()), 64, 1024, 1024, 64, 0, 0, ct.c_void_p(x.data_ptr()),
                                    None)
    assert rc == L.SBR_E_SCRATCH and b"scratch-free" in lib.sbr_last_error()
