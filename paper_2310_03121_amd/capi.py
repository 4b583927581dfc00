"""ctypes declarations of the C ABI in include/nnp.h (argument marshalling only).

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnnp.so")

NNP_OK = 0
STATUS_NAMES = {
    0: "NNP_OK", 1: "NNP_E_INVALID", 2: "NNP_E_SPECIES", 3: "NNP_E_BOX", 4: "NNP_E_CAPACITY",
    5: "NNP_E_OOM", 6: "NNP_E_HIP", 7: "NNP_E_NONFINITE", 8: "NNP_E_WORKSPACE", 9: "NNP_E_BUSY",
}
NNP_MLP_FP32 = 0
NNP_MLP_BF16 = 1


class NNPError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}")


class AevParams(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32), ("rc_rad", C.c_float), ("eta_r", C.c_float),
        ("n_shf_r", C.c_int32), ("shf_r", C.POINTER(C.c_float)),
        ("rc_ang", C.c_float), ("eta_a", C.c_float), ("zeta", C.c_float),
        ("n_shf_a", C.c_int32), ("shf_a", C.POINTER(C.c_float)),
        ("n_shf_z", C.c_int32), ("shf_z", C.POINTER(C.c_float)),
        ("radial_prefactor", C.c_float), ("angle_cos_scale", C.c_float),
    ]


class MlpParams(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("width", C.POINTER(C.c_int32)), ("celu_alpha", C.c_float),
        ("params", C.POINTER(C.c_float)), ("self_energy", C.POINTER(C.c_double)),
    ]


# (name, restype, argtypes)
_P = C.c_void_p
_I = C.c_int32
_SIGS = [
    ("nnp_create", C.c_int, [C.POINTER(AevParams), C.POINTER(MlpParams), C.c_int, C.POINTER(_P)]),
    ("nnp_create_ensemble", C.c_int, [C.POINTER(AevParams), C.POINTER(MlpParams), _I, C.c_int,
                                      C.POINTER(_P)]),
    ("nnp_destroy", None, [_P]),
    ("nnp_param_count", C.c_size_t, [_P]),
    ("nnp_set_params_device", C.c_int, [_P, _P, _P]),
    ("nnp_set_max_neighbors", C.c_int, [_P, _I]),
    ("nnp_set_triclinic", C.c_int, [_P, _I]),
    ("nnp_set_deterministic", C.c_int, [_P, _I]),
    ("nnp_workspace_bytes", C.c_size_t, [_P, _I, _I, _P]),
    ("nnp_energy_forces", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    ("nnp_energy_forces_noalloc", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("nnp_energy_forces_subset", C.c_int, [_P, _I, _I, _P, _I, _P, _P, _P, _P, _P, _P, _P,
                                            C.c_size_t, _P]),
    ("nnp_backward", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    ("nnp_energy_forces_owned", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    ("nnp_check", C.c_int, [_P, _P, _P]),
    ("nnp_status_string", C.c_char_p, [C.c_int]),
    ("nnp_debug_neighbors", C.c_int, [_P, _I, _P, C.c_size_t, _P, _P, _P]),
    ("nnp_debug_aev", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    ("nnp_debug_atom_energies", C.c_int, [_P, _I, _I, _P, _P, C.c_size_t, _P, _P]),
    ("nnp_graph_capture", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P,
                                     C.POINTER(_P)]),
    ("nnp_graph_launch", C.c_int, [_P, _P]),
    ("nnp_graph_destroy", None, [_P]),
    ("nnp_profile_enable", C.c_int, [_P, C.c_int]),
    ("nnp_profile_collect", C.c_int, [_P, _P]),
    ("nnp_profile_stage_count", _I, []),
    ("nnp_profile_stage_name", C.c_char_p, [_I]),
    ("nnp_profile_read", C.c_int, [_P, _P, _P, _I]),
    ("nnp_md_steps", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P, C.c_double, _I, _P, _P,
                                _P, C.c_size_t, _P]),
    ("nnp_langevin_steps", C.c_int, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P, C.c_double, _I,
                                      C.c_double, C.c_double, C.c_uint64, C.c_uint64, _P, _P,
                                      _P, C.c_size_t, _P]),
    ("nnp_server_create", C.c_int, [_P, C.c_size_t, _I, _I, C.c_double, _P, _P, C.POINTER(_P)]),
    ("nnp_server_destroy", None, [_P]),
    ("nnp_server_set_langevin", C.c_int, [_P, C.c_double, C.c_double]),
    ("nnp_server_submit", C.c_int, [_P, C.c_int64, _I, _P, _P, _P, _I]),
    ("nnp_server_step", C.c_int, [_P]),
    ("nnp_server_active", _I, [_P]),
    ("nnp_server_pending", _I, [_P]),
    ("nnp_server_poll", _I, [_P, _P, _I]),
    ("nnp_server_result", C.c_int, [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P]),
    ("nnp_server_stats", C.c_int, [_P, _P, _I]),
]
SYMBOLS = [s[0] for s in _SIGS]

_lib = None


def lib():
    """The loaded engine; raises if libnnp.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP engine not built ({LIB_PATH} missing): run python -m paper_2310_03121_amd.build")
        l = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(l, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def check(code: int, where: str):
    if code != NNP_OK:
        raise NNPError(code, where)
