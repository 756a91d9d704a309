"""ctypes declarations of libqs.so (the C ABI in include/qs.h).

Argument marshalling only: every computation happens in the library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")

QS_OK, QS_EINVAL, QS_ENOMEM, QS_EDEVICE, QS_EUNSUPPORTED = 0, -1, -2, -3, -4
QS_C64, QS_C128 = 0, 1
QS_PLAIN, QS_FUSED = 0, 1
QS_MAX_GATE_WIRES = 6

GATE_KINDS = ["I", "H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SX", "RX", "RY", "RZ", "P", "U",
              "CNOT", "CZ", "CPHASE", "SWAP", "RZZ", "RXX", "RYY", "CU", "MCZ", "MCP", "UNITARY"]
KIND = {k: i for i, k in enumerate(GATE_KINDS)}


class QsGate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nw", C.c_int32), ("wires", C.c_int32 * QS_MAX_GATE_WIRES),
                ("param", C.c_int32), ("reserved", C.c_int32), ("theta", C.c_double),
                ("scale", C.c_double), ("mask", C.c_uint64), ("mat", C.POINTER(C.c_double))]


class QsPauli(C.Structure):
    _fields_ = [("coeff", C.c_double), ("x_mask", C.c_uint64), ("z_mask", C.c_uint64)]


class QsPlanOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_tile_bits", C.c_int32), ("dense_k_max", C.c_int32),
                ("window_k", C.c_int32), ("low_bits", C.c_int32), ("coset_order", C.c_int32),
                ("diag_low_bits", C.c_int32), ("balance_passes", C.c_int32)]


class QsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qs error {code}: {msg}")
        self.code = code


_lib = None

P = C.c_void_p
SZ = C.c_size_t
_SIGS = {
    "qs_last_error": ([], C.c_char_p),
    "qs_version": ([], C.c_char_p),
    "qs_memory_info": ([C.POINTER(SZ), C.POINTER(SZ)], C.c_int),
    "qs_alloc": ([C.c_int, C.c_int, P, P, SZ, P, C.POINTER(P)], C.c_int),
    "qs_free": ([P], C.c_int),
    "qs_state_buffers": ([P, C.POINTER(P), C.POINTER(P)], C.c_int),
    "qs_state_info": ([P, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "qs_set_basis": ([P, C.c_uint64], C.c_int),
    "qs_set_uniform": ([P], C.c_int),
    "qs_upload": ([P, P, SZ], C.c_int),
    "qs_download": ([P, P, SZ], C.c_int),
    "qs_copy": ([P, P], C.c_int),
    "qs_sync": ([P], C.c_int),
    "qs_plan_create": ([C.c_int, C.POINTER(QsGate), SZ, SZ, C.POINTER(QsPlanOpts), C.POINTER(P)], C.c_int),
    "qs_plan_set_params": ([P, C.POINTER(C.c_double), SZ], C.c_int),
    "qs_plan_num_layers": ([P, C.POINTER(SZ)], C.c_int),
    "qs_plan_describe": ([P, C.c_char_p, SZ, C.POINTER(SZ)], C.c_int),
    "qs_plan_free": ([P], C.c_int),
    "qs_plan_inverse": ([P, C.POINTER(P)], C.c_int),
    "qs_apply_layer": ([P, P, SZ, SZ], C.c_int),
    "qs_apply_norm2": ([P, P, C.POINTER(C.c_double)], C.c_int),
    "qs_apply_graph": ([P, P], C.c_int),
    "qs_apply_gates": ([P, C.POINTER(QsGate), SZ, C.POINTER(C.c_double), SZ], C.c_int),
    "qs_expect": ([P, C.POINTER(QsPauli), SZ, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "qs_norm2": ([P, C.POINTER(C.c_double)], C.c_int),
    "qs_overlap": ([P, P, C.POINTER(C.c_double)], C.c_int),
    "qs_infidelity": ([P, P, C.POINTER(C.c_double)], C.c_int),
    "qs_amplitudes": ([P, C.POINTER(C.c_uint64), SZ, P], C.c_int),
    "qs_sample": ([P, C.POINTER(C.c_double), SZ, C.POINTER(C.c_uint64)], C.c_int),
    "qs_sample_noalloc": ([P, C.POINTER(C.c_double), SZ, C.POINTER(C.c_uint64)], C.c_int),
    "qs_marginal": ([P, C.c_uint64, C.POINTER(C.c_double)], C.c_int),
    "qs_adjoint_grad": ([P, P, C.POINTER(QsPauli), SZ, C.POINTER(C.c_double), C.POINTER(C.c_double), SZ],
                        C.c_int),
    "qs_batch_create": ([SZ, C.POINTER(C.c_int), C.POINTER(P), C.c_int, C.c_int, P, C.POINTER(P)], C.c_int),
    "qs_batch_refresh": ([P], C.c_int),
    "qs_batch_run": ([P], C.c_int),
    "qs_batch_expect_diag": ([P, C.POINTER(C.POINTER(QsPauli)), C.POINTER(SZ), C.POINTER(C.c_double)], C.c_int),
    "qs_batch_expect": ([P, C.POINTER(C.POINTER(QsPauli)), C.POINTER(SZ), C.POINTER(C.c_double)], C.c_int),
    "qs_batch_set_observables": ([P, C.POINTER(C.POINTER(QsPauli)), C.POINTER(SZ)], C.c_int),
    "qs_batch_expect_stored": ([P, C.POINTER(C.c_double)], C.c_int),
    "qs_batch_state": ([P, SZ, C.POINTER(P)], C.c_int),
    "qs_batch_free": ([P], C.c_int),
    "qs_profile_enable": ([C.c_int], C.c_int),
    "qs_profile_report": ([C.c_char_p, SZ, C.POINTER(SZ)], C.c_int),
    "qs_profile_reset": ([], C.c_int),
}

EXPORTED = tuple(_SIGS)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2609_19147_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != QS_OK:
        raise QsError(code, lib().qs_last_error().decode())
