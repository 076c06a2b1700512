"""ctypes declarations of the C ABI in include/nnp.h (argument marshalling only).

Loading fails loudly when the HIP library has not been built: there is no
CPU fallback of any kind.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnnp_hip.so")

NNP_OK = 0
STATUS_NAMES = {0: "NNP_OK", 1: "NNP_ERR_ARG", 2: "NNP_ERR_NONFINITE", 3: "NNP_ERR_UNSUPPORTED",
                4: "NNP_ERR_OOM", 5: "NNP_ERR_HIP", 6: "NNP_ERR_STATE"}
DTYPES = {"fp32": 0, "bf16": 1, "fp8": 2, "bf16x3": 3}
PATHS = {"plain": 0, "fused": 1, "split": 2}
RETURN_MODES = {"energy_forces": 3, "energy": 1}

#: Every function the header declares.
EXPORTS = ("nnp_create", "nnp_destroy", "nnp_compute", "nnp_compute_device", "nnp_energy_device",
           "nnp_forces_device", "nnp_energy_device_static", "nnp_set_state",
           "nnp_get_state", "nnp_step", "nnp_capture", "nnp_energy_log", "nnp_stats", "nnp_get_config", "nnp_debug_descriptors",
           "nnp_debug_atom_energies", "nnp_device_bytes", "nnp_autotune", "nnp_time_kernels", "nnp_time_steps",
           "nnp_set_thermostat", "nnp_set_box", "nnp_add_force", "nnp_clear_forces",
           "nnp_debug_fp8_encode",
           "nnp_last_error", "nnp_status_string")


#: nnp_force_fn: (user, n_atoms, n_molecules, d_pos, d_forces, d_energy, stream) -> int
FORCE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32),
        ("n_molecules", ctypes.c_int32),
        ("mol_offsets", ctypes.POINTER(ctypes.c_int32)),
        ("species", ctypes.POINTER(ctypes.c_int32)),
        ("masses", ctypes.POINTER(ctypes.c_double)),
        ("weights", ctypes.POINTER(ctypes.c_float)),
        ("weights_count", ctypes.c_size_t),
        ("mlp_dtype", ctypes.c_int),
        ("path", ctypes.c_int),
        ("return_mode", ctypes.c_int),
        ("rebuild_every", ctypes.c_int32),
        ("skin", ctypes.c_double),
        ("max_neighbors", ctypes.c_int32),
        ("atoms_per_tile", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("use_stream", ctypes.c_int32),
        ("network_tile", ctypes.c_int32),
    ]


class NNPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status
        self.message = message


_lib = None


def _init_torch_first():
    """PyTorch-ROCm wheels carry their own copy of the HIP runtime, so a
    process that uses both PyTorch and this library holds two.  PyTorch's
    must be initialised first (in the other order PyTorch finds no device),
    so it is brought up here, before the library's runtime is loaded,
    whenever PyTorch is importable."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load():
    """Loads libnnp_hip.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library %s is not built; run `python -m paper_2412_18271_amd.build`"
                          % LIB_PATH)
    _init_torch_first()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, d, i32, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64
    st = ctypes.c_int
    sig = {
        "nnp_create": (st, [P(Params), P(vp)]),
        "nnp_destroy": (None, [vp]),
        "nnp_compute": (st, [vp, P(d), P(d), P(d), P(d)]),
        "nnp_compute_device": (st, [vp, vp, ctypes.c_int, vp, vp]),
        "nnp_energy_device": (st, [vp, vp, ctypes.c_int, vp, ctypes.c_int]),
        "nnp_forces_device": (st, [vp, vp]),
        "nnp_energy_device_static": (st, [vp, vp, ctypes.c_int, vp]),
        "nnp_set_state": (st, [vp, P(d), P(d)]),
        "nnp_get_state": (st, [vp, P(d), P(d), P(d), P(d), P(d)]),
        "nnp_step": (st, [vp, d, i32, i32]),
        "nnp_capture": (st, [vp, d, i32]),
        "nnp_energy_log": (st, [vp, i32, P(d), P(d), P(i32)]),
        "nnp_stats": (st, [vp, P(i64)]),
        "nnp_get_config": (st, [vp, P(i32)]),
        "nnp_debug_descriptors": (st, [vp, P(d), P(ctypes.c_float)]),
        "nnp_debug_atom_energies": (st, [vp, P(d)]),
        "nnp_device_bytes": (st, [vp, P(i64)]),
        "nnp_autotune": (st, [vp, ctypes.c_char_p, P(i32)]),
        "nnp_time_kernels": (st, [vp, i32, P(d)]),
        "nnp_time_steps": (st, [vp, d, i32, P(d)]),
        "nnp_set_thermostat": (st, [vp, d, d, ctypes.c_uint64]),
        "nnp_set_box": (st, [vp, P(d)]),
        "nnp_add_force": (st, [vp, FORCE_FN, vp, vp, vp, vp]),
        "nnp_clear_forces": (st, [vp]),
        "nnp_debug_fp8_encode": (st, [P(ctypes.c_float), i32, vp, vp]),
        "nnp_last_error": (ctypes.c_char_p, [vp]),
        "nnp_status_string": (ctypes.c_char_p, [st]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
