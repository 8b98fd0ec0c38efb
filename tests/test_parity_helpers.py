"""CPU checks of the comparison helpers the GPU parity tests use."""
import numpy as np

from paper_2311_13182_amd import scenes as S

from _parity import fd_coords_local, union_flags


def test_local_coordinate_differences_equal_full_recomputation(orc):
    sc = S.icosphere_scene(level=2, n_rays=24, n_chirps=2)
    o = orc.trace(sc)
    tgt, _, _ = orc.forward(S.jitter(sc, 2e-3, 3))
    hit_v = np.unique(sc.faces[np.unique(o["tri"][o["tri"] >= 0])].reshape(-1))
    coords = hit_v[:5] * 3 + np.arange(5) % 3
    loc = fd_coords_local(orc, sc, o["tri"], o["flags"], tgt, coords)
    full = orc.fd_grad(sc, o["tri"], o["flags"], tgt, coords=coords)
    assert np.max(np.abs(loc - full)) <= 1e-6 * np.max(np.abs(full)) and np.max(np.abs(full)) > 0


def test_union_flags_is_bitwise_or():
    a = np.array([[0, 1, 0], [16, 0, 32]], np.uint8)
    b = np.array([[2, 0, 0], [0, 0, 1]], np.uint8)
    assert np.array_equal(union_flags(a, b), a | b)
