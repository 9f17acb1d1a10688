"""ctypes declarations mirroring include/qflex.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqflex.so")

OK, E_INVALID, E_PLAN, E_NOMEM, E_DEVICE, E_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "QFLEX_OK", 1: "QFLEX_E_INVALID", 2: "QFLEX_E_PLAN", 3: "QFLEX_E_NOMEM",
                4: "QFLEX_E_DEVICE", 5: "QFLEX_E_UNSUPPORTED"}
PREC = {"c64": 0, "split_bf16": 1, "split_fp16": 2}
PLAN = {"auto": 0, "sweep": 1, "quadrant": 2, "cut_sweep": 3}
SLICES = {"random": 0, "block": 1}
KIND = {"h": 0, "x12": 1, "y12": 2, "t": 3, "cz": 4, "fsim": 5, "mat1": 6, "mat2": 7}


class Gate(C.Structure):
    _fields_ = [("cycle", C.c_int32), ("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("theta", C.c_double), ("phi", C.c_double), ("mat", C.POINTER(C.c_double))]


class Circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("xy", C.POINTER(C.c_int32)),
                ("gates", C.POINTER(Gate)), ("n_gates", C.c_int64)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("plan_kind", C.c_int32),
                ("max_tensor_elems", C.c_int64), ("open_qubits", C.POINTER(C.c_int32)),
                ("n_open", C.c_int32), ("bitstring_batch", C.c_int32),
                ("slice_mode", C.c_int32), ("graph", C.c_int32), ("autotune", C.c_int32),
                ("fused", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("flops", C.c_double), ("permute_bytes", C.c_double), ("n_gemm", C.c_int64),
                ("n_permute", C.c_int64), ("n_slices", C.c_int64), ("n_bitstrings", C.c_int64),
                ("n_tuned", C.c_int64)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


EXPORTS = ("qflex_build_grid", "qflex_update_gates", "qflex_num_slices", "qflex_plan_cuts", "qflex_plan_describe",
           "qflex_contract_amplitudes", "qflex_contract_grad", "qflex_last_stats",
           "qflex_set_profiling",
           "qflex_profile_read", "qflex_permute_c64", "qflex_gemm_split_c64",
           "qflex_gemm_split_c64_noalloc", "qflex_gemm_split_c64_tile",
           "qflex_gemm_c64", "qflex_select_slices", "qflex_frugal_sample", "qflex_fidelity_samples",
           "qflex_autotune_cache_save", "qflex_autotune_cache_load", "qflex_autotune_cache_size",
           "qflex_autotune_cache_clear",
           "qflex_gemm_split_workspace", "qflex_gemm_c64_workspace", "qflex_gemm_variant",
           "qflex_grid_free", "qflex_last_error")
# exports that do not return a qflex_status, with their return types
# the no-allocation split product's fixed scratch size (QFLEX_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20
NON_STATUS = {"qflex_autotune_cache_size": C.c_int64, "qflex_autotune_cache_clear": None,
              "qflex_gemm_split_workspace": C.c_int64, "qflex_gemm_c64_workspace": C.c_int64,
              "qflex_gemm_variant": C.c_int32, "qflex_grid_free": None,
              "qflex_last_error": C.c_char_p}

_lib = None


def lib():
    """Load libqflex.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libqflex.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1811_09599_amd.build)")
    # One HIP runtime per process: torch ships its own libamdhip64; loading it first makes
    # libqflex bind to that same runtime instead of bringing in a second one, so that device
    # pointers and streams from torch are valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.qflex_build_grid.argtypes = [C.POINTER(Circuit), C.c_int32, C.POINTER(Options), P,
                                   C.POINTER(P)]
    L.qflex_num_slices.argtypes = [P, C.c_int32, C.POINTER(C.c_int64)]
    L.qflex_update_gates.argtypes = [P, C.c_int32, C.POINTER(Circuit), P]
    L.qflex_plan_cuts.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                  C.POINTER(C.c_int32)]
    L.qflex_plan_describe.argtypes = [C.POINTER(Circuit), C.POINTER(Options), C.c_char_p,
                                      C.c_int64, C.POINTER(C.c_int64)]
    L.qflex_contract_amplitudes.argtypes = [P, C.POINTER(C.c_uint8), C.POINTER(C.c_int64),
                                            C.c_double, C.c_uint64, C.POINTER(C.c_int64),
                                            C.POINTER(C.c_int64), P, C.c_int32, P]
    L.qflex_contract_grad.argtypes = [P, C.POINTER(C.c_uint8), C.POINTER(C.c_int64), C.c_double,
                                      C.c_uint64, C.POINTER(C.c_int64), C.POINTER(C.c_int64), P,
                                      C.c_int32, P, P, P, P, C.c_int32, P]
    L.qflex_last_stats.argtypes = [P, C.POINTER(Stats)]
    L.qflex_set_profiling.argtypes = [P, C.c_int32]
    L.qflex_profile_read.argtypes = [P, C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]
    L.qflex_permute_c64.argtypes = [P, P, C.c_int32, C.POINTER(C.c_int32), C.c_int64, P]
    L.qflex_gemm_c64.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                 C.c_int64, P, C.c_int64, P]
    L.qflex_gemm_c64_workspace.argtypes = [C.c_int64] * 4
    L.qflex_gemm_variant.argtypes = [C.c_int64, C.c_int64, C.c_int64]
    L.qflex_select_slices.argtypes = [C.c_int64, C.c_double, C.c_uint64, C.c_int32,
                                      C.POINTER(C.c_int64), C.c_int64, C.POINTER(C.c_int64)]
    L.qflex_frugal_sample.argtypes = [P, C.c_int64, C.c_int64, P, P, C.c_int32, C.c_int32,
                                      C.c_double, P, P, P, P]
    L.qflex_fidelity_samples.argtypes = [P, P, C.c_int64, P, C.c_double, P, P, P, C.c_int32,
                                         C.c_double, P, P, P]
    L.qflex_autotune_cache_save.argtypes = [C.c_char_p]
    L.qflex_autotune_cache_load.argtypes = [C.c_char_p, C.POINTER(C.c_int64)]
    L.qflex_autotune_cache_size.argtypes = []
    L.qflex_autotune_cache_clear.argtypes = []
    L.qflex_grid_free.argtypes = [P]
    L.qflex_gemm_split_c64.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                                       C.c_int32, C.c_int64, C.c_int32, P, C.c_int64, P]
    L.qflex_gemm_split_workspace.argtypes = [C.c_int64] * 4
    L.qflex_gemm_split_c64_noalloc.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64,
                                               C.c_int32, C.c_int32, C.c_int64, C.c_int32, P]
    L.qflex_gemm_split_c64_tile.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64,
                                            C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                            C.c_int32, P, C.c_int64, P]
    for name in EXPORTS:
        getattr(L, name).restype = NON_STATUS.get(name, C.c_int)
    _lib = L
    return L


class QflexError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


def check(status: int):
    if status != OK:
        raise QflexError(status, lib().qflex_last_error().decode())
