"""ctypes declarations of the libsbr C ABI (include/sbr.h).

Argument marshalling only.  The library is the in-tree `libsbr.so` built by
`paper_2311_13182_amd/build.py`; importing this module fails loudly when it is
missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsbr.so")

SBR_OK, SBR_E_ARG, SBR_E_HIP, SBR_E_SCRATCH, SBR_E_UNSUPPORTED = 0, -1, -2, -3, -4
SBR_MAX_BOUNCES, SBR_MAX_TX, SBR_MAX_RX, SBR_MAX_VIRTUAL, SBR_MAX_MATERIALS = 8, 20, 20, 400, 64
SBR_HIT_EDGE, SBR_HIT_TIE, SBR_HIT_GRAZE, SBR_HIT_TMIN, SBR_HIT_PARENT = 1, 2, 4, 8, 16
SBR_HIT_OCCLUDED = 32
SBR_RAYS_SHADOW, SBR_RAYS_JITTER = 1, 2
SBR_DROP_FLAGGED = 1
SBR_ATTACHED = 2
SBR_EXIT_ONLY = 4
SBR_DIRECT_SUMS = 8
SBR_PATHS_IN_SCRATCH = 16
SBR_OP_BUILD_BVH, SBR_OP_SYNTH, SBR_OP_BACKWARD, SBR_OP_RADAR_CUBE, SBR_OP_CFAR = 0, 1, 2, 3, 4
SBR_LOSS_SCRATCH_BYTES = 8192
SBR_MAX_BATCH = 1024
SBR_NOALLOC_SCRATCH_BYTES = 64 << 20

# every function declared in include/sbr.h
EXPORTS = ("sbr_bvh_bytes", "sbr_scratch_bytes", "sbr_build_bvh", "sbr_trace", "sbr_synth_if",
           "sbr_radar_cube", "sbr_cfar", "sbr_backward", "sbr_last_error", "sbr_loss_grad", "sbr_profile",
           "sbr_profile_read", "sbr_radar_cube_2d", "sbr_radar_cube_2d_bytes", "sbr_cloud",
           "sbr_angle_peaks", "sbr_angle_peaks_bytes", "sbr_batch_table_bytes", "sbr_synth_if_batched",
           "sbr_backward_batched", "sbr_radar_cube_noalloc")
PROF_SYNTH, PROF_SYNTH_ADJ, PROF_TRACE, PROF_NU_SPREAD, PROF_NU_TAPS = 0, 1, 2, 3, 4


class SbrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsbr error {code}: {msg}")
        self.code = code


class sbr_mesh(ct.Structure):
    _fields_ = [("verts", ct.c_void_p), ("nv", ct.c_int32), ("faces", ct.c_void_p), ("nf", ct.c_int32),
                ("mat_id", ct.c_void_p)]


class sbr_material(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("reserved", ct.c_int32), ("eps_r", ct.c_double), ("sigma", ct.c_double)]


class sbr_radar(ct.Structure):
    _fields_ = [("origin", ct.c_double * 3), ("rot", ct.c_double * 9), ("n_tx", ct.c_int32),
                ("n_rx", ct.c_int32), ("tx", (ct.c_double * 3) * SBR_MAX_TX),
                ("rx", (ct.c_double * 3) * SBR_MAX_RX), ("velocity", ct.c_double * 3),
                ("attenuation", ct.c_double), ("tx_gain_exp", ct.c_double), ("rx_gain_exp", ct.c_double)]


class sbr_chirp(ct.Structure):
    _fields_ = [("fc", ct.c_double), ("slope", ct.c_double), ("fs", ct.c_double), ("t_chirp", ct.c_double),
                ("n_samples", ct.c_int32), ("n_chirps", ct.c_int32)]


class sbr_rays(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("tan_half_x", ct.c_double),
                ("tan_half_y", ct.c_double), ("max_bounces", ct.c_int32), ("options", ct.c_int32),
                ("t_min", ct.c_double), ("seed_lo", ct.c_uint32), ("seed_hi", ct.c_uint32)]


class sbr_param_grads(ct.Structure):
    _fields_ = [("materials", ct.c_void_p), ("radar", ct.c_void_p), ("rot", ct.c_void_p),
                ("attenuation", ct.c_void_p)]


class sbr_hits(ct.Structure):
    _fields_ = [("tri", ct.c_void_p), ("t", ct.c_void_p), ("u", ct.c_void_p), ("v", ct.c_void_p),
                ("flags", ct.c_void_p)]


class sbr_request(ct.Structure):
    _fields_ = [("mesh", ct.POINTER(sbr_mesh)), ("mats", ct.POINTER(sbr_material)), ("n_mats", ct.c_int32),
                ("flags", ct.c_int32), ("radar", ct.POINTER(sbr_radar)), ("rays", ct.POINTER(sbr_rays)),
                ("hits", ct.POINTER(sbr_hits)), ("chirp", ct.POINTER(sbr_chirp)), ("if_cube", ct.c_void_p),
                ("grad_if", ct.c_void_p), ("grad_verts", ct.c_void_p), ("params", ct.POINTER(sbr_param_grads)),
                ("scratch", ct.c_void_p), ("scratch_bytes", ct.c_size_t)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libsbr.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libsbr.so not found at {path}; build it with "
                          f"`python -m paper_2311_13182_amd.build` (hipcc, gfx950)")
    # The library shares device memory and streams with PyTorch, so it must bind
    # to the HIP runtime PyTorch loads: import torch before the library.
    import torch  # noqa: F401
    L = ct.CDLL(path)
    P = ct.POINTER
    vp, i32, sz = ct.c_void_p, ct.c_int32, ct.c_size_t
    L.sbr_last_error.restype = ct.c_char_p
    L.sbr_last_error.argtypes = []
    L.sbr_bvh_bytes.restype = sz
    L.sbr_bvh_bytes.argtypes = [i32]
    L.sbr_scratch_bytes.restype = sz
    L.sbr_scratch_bytes.argtypes = [i32, P(sbr_mesh), P(sbr_rays), P(sbr_radar), P(sbr_chirp)]
    L.sbr_build_bvh.restype = ct.c_int
    L.sbr_build_bvh.argtypes = [P(sbr_mesh), vp, sz, i32, vp, sz, vp]
    L.sbr_trace.restype = ct.c_int
    L.sbr_trace.argtypes = [P(sbr_mesh), vp, P(sbr_radar), P(sbr_rays), P(sbr_hits), vp, vp]
    L.sbr_synth_if.restype = ct.c_int
    L.sbr_synth_if.argtypes = [P(sbr_mesh), P(sbr_material), i32, P(sbr_radar), P(sbr_rays), P(sbr_hits),
                               P(sbr_chirp), i32, vp, vp, sz, vp]
    L.sbr_radar_cube.restype = ct.c_int
    L.sbr_radar_cube.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp, sz, vp]
    L.sbr_radar_cube_2d.restype = ct.c_int
    L.sbr_radar_cube_2d.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i32, vp, vp, sz, vp]
    L.sbr_angle_peaks.restype = ct.c_int
    L.sbr_angle_peaks.argtypes = [vp, i32, i32, i32, i32, vp, vp, i32, ct.c_float, vp, i32, vp, vp, sz, vp]
    L.sbr_angle_peaks_bytes.restype = sz
    L.sbr_angle_peaks_bytes.argtypes = [i32, i32, i32]
    L.sbr_cloud.restype = ct.c_int
    L.sbr_cloud.argtypes = [vp, vp, i32, P(sbr_radar), P(sbr_chirp), i32, i32, vp, vp]
    L.sbr_radar_cube_2d_bytes.restype = sz
    L.sbr_radar_cube_2d_bytes.argtypes = [i32, i32, i32, i32, i32, i32]
    L.sbr_cfar.restype = ct.c_int
    L.sbr_cfar.argtypes = [vp, i32, i32, i32, i32, i32, ct.c_double, vp, vp, i32, vp, vp, sz, vp]
    L.sbr_backward.restype = ct.c_int
    L.sbr_backward.argtypes = [P(sbr_mesh), P(sbr_material), i32, P(sbr_radar), P(sbr_rays), P(sbr_hits),
                               P(sbr_chirp), i32, vp, vp, P(sbr_param_grads), vp, sz, vp]
    L.sbr_loss_grad.restype = ct.c_int
    L.sbr_loss_grad.argtypes = [i32, vp, vp, ct.c_int64, vp, vp, vp, sz, vp]
    L.sbr_profile.restype = ct.c_int
    L.sbr_profile.argtypes = [i32]
    L.sbr_profile_read.restype = ct.c_int
    L.sbr_profile_read.argtypes = [i32, P(ct.c_double), P(ct.c_int64)]
    L.sbr_batch_table_bytes.restype = sz
    L.sbr_batch_table_bytes.argtypes = [i32]
    L.sbr_synth_if_batched.restype = ct.c_int
    L.sbr_synth_if_batched.argtypes = [P(sbr_request), i32, vp, sz, vp]
    L.sbr_backward_batched.restype = ct.c_int
    L.sbr_backward_batched.argtypes = [P(sbr_request), i32, vp, sz, vp]
    L.sbr_radar_cube_noalloc.restype = ct.c_int
    L.sbr_radar_cube_noalloc.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp]
    _lib = L
    return L


def check(rc: int):
    if rc != SBR_OK:
        raise SbrError(rc, load().sbr_last_error().decode())
    return rc
