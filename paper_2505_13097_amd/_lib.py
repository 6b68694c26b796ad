"""ctypes declarations of the C ABI in include/lbm_stefan.h.

torch is imported before the library is loaded: the library links the HIP
runtime by soname, and with torch already loaded the process keeps a
single HIP runtime shared by both (same device context, same streams).
"""
import ctypes
import os

import torch  # noqa: F401  (must be loaded first, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_stefan.so")

OK, EINVAL, EDEVICE, ENOTCONV, ENAN = 0, -1, -2, -3, -4
BC_DIRICHLET, BC_BOUNCEBACK, BC_PERIODIC, BC_NEUMANN = 0, 1, 2, 3
STORE_F64, STORE_F32 = 0, 1
NEWTON_SAFEGUARDED, NEWTON_PLAIN = 0, 1
FRONT_LIQUID_INTEGRAL, FRONT_ZERO_CROSSING = 0, 1
FIELD_T, FIELD_STATE, FIELD_LIQUID = 0, 1, 2
FLAG_ADJOINT, FLAG_CHECKED_FACES = 1, 2
SCHEME_IREBM, SCHEME_EEBM, SCHEME_ILFBM = 0, 1, 2

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("q", ctypes.c_int32),
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("storage", ctypes.c_int32), ("newton_mode", ctypes.c_int32),
        ("tau", ctypes.c_double), ("ste", ctypes.c_double),
        ("t_m", ctypes.c_double), ("delta", ctypes.c_double),
        ("bc", ctypes.c_int32 * 4), ("wall_T", ctypes.c_double * 4),
        ("wall_profile", _c_double_p * 4),
        ("dx", ctypes.c_double), ("newton_tol", ctypes.c_double),
        ("newton_max_it", ctypes.c_int32), ("strict", ctypes.c_int32),
        ("variant", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("nz", ctypes.c_int64), ("bc_z", ctypes.c_int32 * 2),
        ("wall_T_z", ctypes.c_double * 2),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("max_newton_it", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("nonconverged", ctypes.c_int64),
        ("max_residual", ctypes.c_double), ("energy", ctypes.c_double),
        ("flux_in", ctypes.c_double), ("flux_out", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_
                if k != "reserved"}


# name -> (restype, argtypes)
_vp = ctypes.c_void_p
_P = ctypes.POINTER(Params)
SIGNATURES = {
    "lbm_stefan_version": (ctypes.c_char_p, []),
    "lbm_stefan_last_error": (ctypes.c_char_p, [_vp]),
    "lbm_stefan_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_stefan_init": (ctypes.c_int, [_P, _c_double_p, _vp, ctypes.c_size_t, _vp,
                                       ctypes.POINTER(_vp)]),
    "lbm_stefan_step": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.POINTER(Stats)]),
    "lbm_stefan_reset_stats": (ctypes.c_int, [_vp]),
    "lbm_stefan_query_front": (ctypes.c_int, [_vp, ctypes.c_int32, _c_double_p,
                                              _c_double_p]),
    "lbm_stefan_get_field": (ctypes.c_int, [_vp, ctypes.c_int32, _vp]),
    "lbm_stefan_set_state": (ctypes.c_int, [_vp, _vp, ctypes.c_int32]),
    "lbm_stefan_state_ptr": (ctypes.c_int, [_vp, ctypes.POINTER(_vp)]),
    "lbm_stefan_variant_count": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int32)]),
    "lbm_stefan_variant_name": (ctypes.c_char_p, [ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32]),
    "lbm_stefan_set_variant": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "lbm_stefan_autotune": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32),
                                           _c_double_p]),
    "lbm_stefan_destroy": (ctypes.c_int, [_vp]),
    "lbm_stefan_step_noalloc": (ctypes.c_int, [_P, _vp, _vp, ctypes.POINTER(Stats),
                                                _vp]),
    "lbm_stefan_adjoint_reset": (ctypes.c_int, [_vp]),
    "lbm_stefan_front_vjp": (ctypes.c_int, [_vp, _vp, _c_double_p, _vp]),
    "lbm_stefan_adjoint_step": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_stefan_adjoint_initial_state": (ctypes.c_int, [_vp, _vp]),
    "lbm_stefan_adjoint_gradients": (ctypes.c_int, [_vp, _c_double_p, _c_double_p,
                                                    _c_double_p]),
    "lbm_stefan_adjoint_buffers": (ctypes.c_int, [_vp, ctypes.POINTER(_vp),
                                                  ctypes.POINTER(_vp)]),
    "lbm_stefan_tape_bytes": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_stefan_forward_tape": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64,
                                               _vp, ctypes.c_size_t]),
    "lbm_stefan_backward_tape": (ctypes.c_int, [_vp, _c_double_p, _vp,
                                                ctypes.c_size_t, _c_double_p,
                                                _c_double_p, _c_double_p]),
    "lbm_stefan_batch_workspace_bytes": (ctypes.c_int, [_P, ctypes.c_int32,
                                                        ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_stefan_batch_init": (ctypes.c_int, [_P, ctypes.c_int32,
                                             ctypes.POINTER(_c_double_p), _vp,
                                             ctypes.c_size_t, _vp,
                                             ctypes.POINTER(_vp)]),
    "lbm_stefan_batch_set_schedule": (ctypes.c_int, [_vp, ctypes.c_int32,
                                                     ctypes.c_int32, ctypes.c_int32]),
    "lbm_stefan_batch_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lbm_stefan_batch_stats": (ctypes.c_int, [_vp, ctypes.POINTER(Stats)]),
    "lbm_stefan_batch_reset_stats": (ctypes.c_int, [_vp]),
    "lbm_stefan_batch_query_front": (ctypes.c_int, [_vp, ctypes.c_int32,
                                                    ctypes.c_int32, _c_double_p,
                                                    _c_double_p]),
    "lbm_stefan_batch_get_field": (ctypes.c_int, [_vp, ctypes.c_int32,
                                                  ctypes.c_int32, _vp]),
    "lbm_stefan_batch_state_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_stefan_batch_autotune": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t,
                                                 ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32),
                                                 _c_double_p]),
    "lbm_stefan_batch_last_error": (ctypes.c_char_p, [_vp]),
    "lbm_stefan_batch_destroy": (ctypes.c_int, [_vp]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded library.  Raises LibraryMissing if it was never built:
    there is no CPU fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is not built: run `python __graft_entry__.py` "
                "or paper_2505_13097_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm_stefan error {code}: {msg}")
        self.code = code


def check(rc, handle=None):
    if rc != OK:
        msg = lib().lbm_stefan_last_error(handle)
        raise LbmError(rc, msg.decode() if msg else "")


def check_batch(rc, batch=None):
    if rc != OK:
        msg = lib().lbm_stefan_batch_last_error(batch)
        raise LbmError(rc, msg.decode() if msg else "")
