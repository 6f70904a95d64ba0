"""ctypes declarations of the C ABI in include/sv.h (argument marshalling only).

The shared library must exist: there is no fallback.  Build it with
``python -m paper_2111_06868_amd.build_lib`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsv.so")

SV_MAX_K = 6

OK = 0
ERR_ARG = -1
ERR_QUBIT = -2
ERR_SIZE = -3
ERR_HIP = -4
ERR_UNSUPPORTED = -5

C64 = 0
C128 = 1

PREC_FP32 = 0
PREC_SPLIT_BF16 = 1
PREC_SPLIT_FP16 = 2
PREC_FP64 = 3
PREC_SPLIT_BF16X3 = 4

RULE_PAPER = 0
RULE_ENHANCED = 1
RULE_NONE = 2
RULE_TILED = 3
RULE_AUTO = 4

POP_RIGHT = 0
POP_LEFT = 1

GATE_KINDS = {
    "MATRIX": 0, "I": 1, "X": 2, "Y": 3, "Z": 4, "H": 5, "SQRT_X": 6, "SQRT_Y": 7,
    "SQRT_W": 8, "RX": 9, "RY": 10, "RZ": 11, "CZ": 12, "CX": 13, "CPHASE": 14,
    "SWAP": 15, "FSIM": 16,
}


class sv_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32),
                ("q", ctypes.c_int32 * SV_MAX_K), ("params", ctypes.c_double * 2),
                ("param", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("m", ctypes.POINTER(ctypes.c_double))]


class sv_pauli_sum(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("coef", ctypes.POINTER(ctypes.c_double)),
                ("xmask", ctypes.POINTER(ctypes.c_uint64)),
                ("zmask", ctypes.POINTER(ctypes.c_uint64))]


class sv_run_opts(ctypes.Structure):
    _fields_ = [("max_k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class sv_batch_desc(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int32), ("max_k", ctypes.c_int32),
                ("n_qubits", ctypes.POINTER(ctypes.c_int32)),
                ("gate_offsets", ctypes.POINTER(ctypes.c_int64)),
                ("gates", ctypes.POINTER(sv_gate)), ("precision", ctypes.c_int32)]


class sv_super_op(ctypes.Structure):
    _fields_ = [("after", ctypes.c_int32), ("k", ctypes.c_int32), ("q", ctypes.c_int32 * 3),
                ("n_left", ctypes.c_int32), ("n_right", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("left", ctypes.POINTER(ctypes.c_double)), ("right", ctypes.POINTER(ctypes.c_double)),
                ("s", ctypes.POINTER(ctypes.c_double)), ("superop", ctypes.POINTER(ctypes.c_double))]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.POINTER(ctypes.c_double)
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_GP = ctypes.POINTER(sv_gate)
_PS = ctypes.POINTER(sv_pauli_sum)
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "sv_last_error": (ctypes.c_char_p, []),
    "sv_version": (_I, []),
    "sv_alloc": (_I, [_I, _I, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "sv_free": (_I, [_P]),
    "sv_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_P)]),
    "sv_set_product": (_I, [_P, ctypes.c_char_p]),
    "sv_set_basis": (_I, [_P, _U64]),
    "sv_read": (_I, [_P, _U64, _U64, _P]),
    "sv_write": (_I, [_P, _U64, _U64, _P]),
    "sv_copy": (_I, [_P, _P]),
    "sv_synchronize": (_I, [_P]),
    "sv_gate_matrix": (_I, [_GP, _D]),
    "sv_apply_gate": (_I, [_P, _GP]),
    "sv_fuse": (_I, [_GP, _I, _I, _I, _I, ctypes.POINTER(_P)]),
    "sv_fuse_prec": (_I, [_GP, _I, _I, _I, _I, _I, ctypes.POINTER(_P)]),
    "sv_plan_free": (_I, [_P]),
    "sv_plan_num_blocks": (_I, [_P, ctypes.POINTER(_I)]),
    "sv_plan_block": (_I, [_P, _I, _I32P, _I32P, _I32P]),
    "sv_plan_block_members": (_I, [_P, _I, _I32P]),
    "sv_plan_block_pass": (_I, [_P, _I, _I32P]),
    "sv_plan_block_matrix": (_I, [_P, _I, _D]),
    "sv_plan_max_k": (_I, [_P, ctypes.POINTER(_I)]),
    "sv_plan_rule": (_I, [_P, ctypes.POINTER(_I)]),
    "sv_apply_plan": (_I, [_P, _P, _I, _I]),
    "sv_run_circuit": (_I, [_P, _GP, _I, ctypes.POINTER(sv_run_opts)]),
    "sv_run_circuit_basis": (_I, [_P, ctypes.c_uint64, _GP, _I, ctypes.POINTER(sv_run_opts)]),
    "sv_norm": (_I, [_P, _D]),
    "sv_inner": (_I, [_P, _P, _D, _D]),
    "sv_expectation": (_I, [_P, _PS, _D]),
    "sv_expectation_noalloc": (_I, [_P, _I, _I, _P, _PS, _D]),
    "sv_apply_pauli_sum": (_I, [_P, _PS, _P]),
    "sv_backward": (_I, [_P, _P, _GP, _I, _PS, _D, _I]),
    "sv_backward_prec": (_I, [_P, _P, _GP, _I, _PS, _D, _I, _I]),
    "sv_super_op_matrix": (_I, [ctypes.POINTER(sv_super_op), _D]),
    "sv_dm_run": (_I, [_P, _GP, _I, ctypes.POINTER(sv_super_op), _I, ctypes.POINTER(sv_run_opts)]),
    "sv_dm_expectation": (_I, [_P, _PS, _D]),
    "sv_kraus_probabilities": (_I, [_P, ctypes.POINTER(sv_super_op), _D]),
    "sv_apply_kraus_sampled": (_I, [_P, ctypes.POINTER(sv_super_op), ctypes.c_double, _I32P, _D]),
    "sv_run_trajectory": (_I, [_P, _GP, _I, ctypes.POINTER(sv_super_op), _I, _D,
                               ctypes.POINTER(sv_run_opts), _I32P]),
    "sv_channel_depolarizing": (_I, [_I, _I32P, ctypes.c_double, _I, _D, ctypes.POINTER(sv_super_op)]),
    "sv_channel_dephasing": (_I, [_I, _I, ctypes.c_double, _I, _D, ctypes.POINTER(sv_super_op)]),
    "sv_channel_amplitude_damping": (_I, [_I, ctypes.c_double, ctypes.c_double, _I, _D,
                                          ctypes.POINTER(sv_super_op)]),
    "sv_channel_pauli": (_I, [_I, _I32P, _D, _I, _D, ctypes.POINTER(sv_super_op)]),
    "sv_kraus_form": (_I, [ctypes.POINTER(sv_super_op), _D, ctypes.POINTER(sv_super_op)]),
    "sv_batch_required_bytes": (_I, [ctypes.POINTER(sv_batch_desc), ctypes.POINTER(_SZ)]),
    "sv_batch_create": (_I, [ctypes.POINTER(sv_batch_desc), _P, _SZ, _P, ctypes.POINTER(_P)]),
    "sv_batch_run": (_I, [_P, _I, _D]),
    "sv_batch_read": (_I, [_P, _I, _U64, _U64, _P]),
    "sv_batch_free": (_I, [_P]),
    "sv_autotune": (_I, [_P, _I, _D]),
    "sv_set_cost_table": (_I, [_I, _I, _D]),
    "sv_tune_cache_load": (_I, [ctypes.c_char_p, ctypes.POINTER(_I)]),
    "sv_set_tile_shape": (_I, [_I, _I]),
    "sv_set_tile_union": (_I, [_I]),
    "sv_get_tile_shape": (_I, [ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "sv_tile_placement": (_I, [_I, _I32P, _I, _I, _I, _I, _I32P, ctypes.POINTER(ctypes.c_uint32), _I32P]),
    "sv_project": (_I, [_P, _I, _I32P, _U64, _I, _D]),
    "sv_measure": (_I, [_P, _I, _I32P, _D, ctypes.POINTER(_U64), _D]),
    "sv_controlled_gate": (_I, [_GP, _I, _I32P, _GP, _D]),
    "sv_lightcone": (_I, [_GP, _I, _I, _U64, _I, _I32P, ctypes.POINTER(_I)]),
    "sv_compact_qubits": (_I, [_GP, _I, _I, _U64, _GP, _I32P, ctypes.POINTER(_I)]),
    "sv_simplify": (_I, [_GP, _I, _I, _I, _I32P, ctypes.POINTER(_I)]),
    "sv_stream_probe": (_I, [_P, _U64, _I, _D]),
    "sv_stats_enable": (_I, [_I]),
    "sv_graph_stats": (_I, [_P, _I64P, _I64P]),
    "sv_stats_reset": (_I, []),
    "sv_stats_query": (_I, [_I, _I64P, _D]),
}

_lib = None


class SvError(RuntimeError):
    """A failing sv_* call (SV_ERR_HIP, SV_ERR_UNSUPPORTED, ...)."""

    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class SvValueError(SvError, ValueError):
    """SV_ERR_ARG / SV_ERR_QUBIT / SV_ERR_SIZE: invalid input (the paper's
    circuits raise ValueError on unsupported input, Circuits section)."""


def lib():
    """The loaded libsv.so; raises loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsv.so is not built (%s); run paper_2111_06868_amd.build_lib.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc == OK:
        return
    msg = lib().sv_last_error().decode(errors="replace")
    if rc in (ERR_ARG, ERR_QUBIT, ERR_SIZE):
        raise SvValueError(rc, msg)
    raise SvError(rc, msg)
