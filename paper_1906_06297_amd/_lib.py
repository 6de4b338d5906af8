"""ctypes binding of libising.so (the C ABI declared in include/ising.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI.  If the built library is missing this raises; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libising.so")

ISING_OK = 0
RULE_METROPOLIS, RULE_HEATBATH = 0, 1
ISING_E_BADARG = -1
ISING_E_SIZE = -2
ISING_E_HIP = -3


class IsingError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"ising error {code}: {message}")
        self.code = code


class LatticeStruct(ctypes.Structure):
    _fields_ = [
        ("words", ctypes.c_void_p),
        ("L", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_dbl = ctypes.c_double
_lat_p = ctypes.POINTER(LatticeStruct)

# name -> (restype, argtypes); mirrors include/ising.h
SIGNATURES = {
    "ising_words_per_colour": (_i64, [_i64]),
    "ising_thresholds": (ctypes.c_int, [_dbl, _dbl, ctypes.POINTER(_u64)]),
    "ising_init": (ctypes.c_int, [_lat_p, _vp, ctypes.c_size_t, _i64, _u64, _u32, _vp]),
    "ising_sweep": (ctypes.c_int, [_lat_p, _dbl, _dbl, _i64, _u64, _vp]),
    "ising_glass_bonds_init": (ctypes.c_int, [_vp, ctypes.c_size_t, _i64, _u64, ctypes.c_uint32, _vp]),
    "ising_glass_set_bonds": (ctypes.c_int, [_vp, ctypes.c_size_t, _i64, _vp, _vp, _vp]),
    "ising_glass_sweep": (ctypes.c_int, [_lat_p, _vp, ctypes.c_size_t, _dbl, _dbl, _i64, _u64, _vp]),
    "ising_glass_observables": (ctypes.c_int, [_lat_p, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    "ising_mm_lattice_bytes": (_i64, [_i64]),
    "ising_mm_sums_bytes": (_i64, [_i64]),
    "ising_mm_from_words": (ctypes.c_int, [_lat_p, _vp, ctypes.c_size_t, _vp]),
    "ising_mm_to_words": (ctypes.c_int, [_lat_p, _vp, ctypes.c_size_t, _vp]),
    "ising_mm_sweep": (ctypes.c_int, [_i64, _u64, _u32, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t,
                                      _dbl, _dbl, _i64, _u64, ctypes.c_int, _vp]),
    "ising_thresholds_rule": (ctypes.c_int, [_dbl, _dbl, ctypes.c_int, ctypes.POINTER(_u64)]),
    "ising_sweep_rule": (ctypes.c_int, [_lat_p, _dbl, _dbl, ctypes.c_int, _i64, _u64, _vp]),
    "ising_sweep_traced": (ctypes.c_int, [_lat_p, _dbl, _dbl, _i64, _u64, _vp, _vp, _vp]),
    "ising_observables": (ctypes.c_int, [_lat_p, _vp, _vp, _vp]),
    "ising_get_spins": (ctypes.c_int, [_lat_p, _vp, _vp]),
    "ising_set_spins": (ctypes.c_int, [_lat_p, _vp, _vp]),
    "ising_batch_words": (_i64, [ctypes.c_int32, ctypes.POINTER(_i64)]),
    "ising_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(_i64),
                                          ctypes.POINTER(_dbl), _dbl, ctypes.POINTER(_u64),
                                          ctypes.POINTER(_u32), _vp, ctypes.c_size_t]),
    "ising_batch_destroy": (ctypes.c_int, [_vp]),
    "ising_batch_lattice": (ctypes.c_int, [_vp, ctypes.c_int32, _lat_p]),
    "ising_batch_init": (ctypes.c_int, [_vp, _vp]),
    "ising_batch_sweep": (ctypes.c_int, [_vp, _i64, _vp]),
    "ising_batch_set_counter": (ctypes.c_int, [_vp, _u64, _vp]),
    "ising_batch_get_counter": (ctypes.c_int, [_vp, ctypes.POINTER(_u64), _vp]),
    "ising_batch_observables": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ising_batch_get_tiles": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(_u32),
                                             ctypes.POINTER(_u32)]),
    "ising_batch_set_tiles": (ctypes.c_int, [_vp, _i64, _u32, _u32]),
    "ising_batch_get_plan": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(_u32),
                                            ctypes.POINTER(_u32)]),
    "ising_batch_get_mixed": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "ising_batch_set_bundles": (ctypes.c_int, [_vp, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_int32)]),
    "ising_batch_autotune": (ctypes.c_int, [_vp, _i64, ctypes.c_char_p, _vp]),
    "ising_batch_get_spins_dev": (ctypes.c_int, [_vp, _vp, _vp]),
    "ising_batch_set_spins_dev": (ctypes.c_int, [_vp, _vp, _vp]),
    "ising_philox_rate": (ctypes.c_int, [_u64, _u32, _u64, _u32, _u64, _vp, _u32, _vp]),
    "ising_batch_sweep_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_i64),
                                                 ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                                 ctypes.POINTER(_u64), ctypes.POINTER(_u32), _vp,
                                                 ctypes.c_size_t, _i64, _u64, _vp]),
    "ising_arnet_num_params": (_i64, [ctypes.c_int32]),
    "ising_arnet_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32]),
    "ising_arnet_destroy": (ctypes.c_int, [_vp]),
    "ising_arnet_set_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "ising_arnet_get_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "ising_arnet_log_prob": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "ising_arnet_set_eval_mode": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ising_arnet_gradient": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "ising_arnet_train_step": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_float, _vp, _vp]),
    "ising_arnet_adam": (ctypes.c_int, [_vp, _vp, ctypes.c_float, _vp]),
    "ising_arnet_gradient_at": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "ising_arnet_sample": (ctypes.c_int, [_vp, ctypes.c_int32, _u64, _u32, _u64, _vp, _vp, _vp]),
    "ising_spins_minibatch": (ctypes.c_int, [_vp, _i64, _i64, ctypes.c_int32, _u64, _u32, _u64,
                                             _vp, _vp]),
    "ising_spins_observables": (ctypes.c_int, [_vp, ctypes.c_int32, _i64, _vp, _vp, _vp]),
    "ising_mh_independence": (ctypes.c_int, [ctypes.c_int32, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _u64, _u32, _u64, _vp, _vp]),
    "ising_set_sweep_kernel": (ctypes.c_int, [ctypes.c_int]),
    "ising_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libising.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_1906_06297_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != ISING_OK:
        msg = load().ising_last_error().decode(errors="replace")
        raise IsingError(code, msg)
