"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the method runs in the HIP library libpaper_lbm.so.  torch is
imported before the library is loaded so both use the same HIP runtime; torch
supplies device memory (the population workspace) and the stream.
"""
import ctypes
import os

import torch  # noqa: F401  (must be loaded before the HIP library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpaper_lbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_ECAPACITY, LBM_EUNSTABLE = range(7)
STATUS_NAMES = {0: "LBM_OK", 1: "LBM_EINVAL", 2: "LBM_ENOMEM", 3: "LBM_EDEVICE", 4: "LBM_ESTATE",
                5: "LBM_ECAPACITY", 6: "LBM_EUNSTABLE"}
PSTATE = 10
AGRAD = 25
STORE_F64, STORE_F32, STORE_F16S = 0, 1, 2

_dp = ctypes.POINTER(ctypes.c_double)


class ChannelConfig(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("u_wall", (ctypes.c_double * 2) * 4), ("init", ctypes.c_int32),
        ("body_force", ctypes.c_double * 2), ("gravity", ctypes.c_double * 2),
        ("storage", ctypes.c_int32), ("fp16_exp", ctypes.c_int32),
        ("mls_rw", ctypes.c_double), ("mls_alpha", ctypes.c_double), ("probe_dn", ctypes.c_double),
        ("mls_kernel", ctypes.c_int32), ("spread_scale", ctypes.c_int32),
    ]


class ParticleDesc(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_double), ("y", ctypes.c_double), ("theta", ctypes.c_double),
        ("u", ctypes.c_double), ("v", ctypes.c_double), ("omega", ctypes.c_double),
        ("density_ratio", ctypes.c_double), ("area", ctypes.c_double),
        ("polar_moment", ctypes.c_double), ("n_markers", ctypes.c_int32),
        ("xi", _dp), ("nrm", _dp), ("ds", _dp),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("rows_per_thread", ctypes.c_int32),
                ("persistent_wgs", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("overlap", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("nt_store", ctypes.c_int32), ("adj_fused", ctypes.c_int32)]


# name -> (restype, argtypes); the list mirrors include/lbm.h
SIGNATURES = {
    "lbm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ChannelConfig), ctypes.c_int32]),
    "lbm_init": (ctypes.c_int, [ctypes.POINTER(ChannelConfig), ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_add_particle": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ParticleDesc),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "lbm_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "lbm_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "lbm_get_particles": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_get_fields": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp, _dp, _dp]),
    "lbm_get_fields_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp, _dp, _dp]),
    "lbm_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "lbm_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "lbm_checkpoint_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbm_checkpoint_restore": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbm_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "lbm_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "lbm_time_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "lbm_adjoint_begin": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_int32]),
    "lbm_adjoint_segment": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "lbm_adjoint_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "lbm_adjoint_gradients": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp]),
    "lbm_adjoint_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "lbm_measure_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                        ctypes.c_void_p, _dp]),
    "lbm_adjoint_position": (ctypes.c_int64, [ctypes.c_void_p]),
    "lbm_steps_done": (ctypes.c_int64, [ctypes.c_void_p]),
    "lbm_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "lbm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "(the GPU path has no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, handle=None):
    if code != LBM_OK:
        msg = lib().lbm_last_error(handle)
        raise LBMError(code, msg.decode() if msg else "")
