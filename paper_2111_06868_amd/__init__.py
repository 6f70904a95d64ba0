"""MI355X (gfx950) state-vector simulation: Python binding of libsv.so.

This module only marshals arguments: every step of the path (gate matrices,
fusion, application, reductions, gradients, batches) runs inside the C ABI
library (include/sv.h).  PyTorch provides device memory (a tensor holds each
state) and the HIP stream.  There is no CPU fallback: without the built
library every call raises.

Circuits follow the paper's statement (Circuits section): an ordered list of
gates acting on qubits.  Gates are given on qubit POSITIONS (bit p of the
amplitude index); ``positions(order, qubits)`` maps the paper's named qubits
with an ``order`` list (order[0] = most significant) onto positions.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import _native as N
from ._native import (C64, C128, PREC_FP32, PREC_SPLIT_BF16, PREC_SPLIT_FP16, PREC_FP64,  # noqa: F401
                      PREC_SPLIT_BF16X3,
                      RULE_PAPER, RULE_ENHANCED, RULE_NONE, RULE_TILED, RULE_AUTO, SV_MAX_K, GATE_KINDS, SvError,
                      SvValueError)

__all__ = ["State", "Plan", "fuse", "gate_matrix", "backward", "Energy", "Batch", "positions",
           "DensityMatrix", "SuperOp", "depolarizing", "dephasing", "amplitude_damping", "pauli_channel",
           "local_channels", "kraus_form", "lightcone", "compact_qubits", "simplify", "expectation_noalloc",
           "controlled",
           "pauli_sum", "autotune", "set_cost_table", "tune_cache_load", "set_tile_shape", "get_tile_shape", "set_tile_union", "TILE_SHAPES",
           "stats_enable", "stats_reset", "stats_query",
           "C64", "C128", "PREC_FP32", "PREC_SPLIT_BF16", "PREC_SPLIT_FP16", "PREC_FP64", "PREC_SPLIT_BF16X3",
           "RULE_PAPER", "RULE_ENHANCED", "RULE_NONE", "RULE_TILED", "RULE_AUTO", "SvError", "SvValueError"]


def positions(order: Sequence, qubits: Sequence) -> tuple:
    """Named qubits -> positions: axis j of the paper's (2,)*n array follows
    order[j] (C order), so order[0] is position n-1."""
    n = len(order)
    idx = {q: j for j, q in enumerate(order)}
    return tuple(n - 1 - idx[q] for q in qubits)


# ------------------------------------------------------------------ gates
class GateArray:
    """A ctypes sv_gate[] plus the matrices it points to."""

    def __init__(self, gates):
        gates = list(gates)
        self.n = len(gates)
        self.arr = (N.sv_gate * max(self.n, 1))()
        self._keep = []
        for i, g in enumerate(gates):
            name, qubits, params, param_index, matrix = _gate_fields(g)
            s = self.arr[i]
            if name not in GATE_KINDS:
                raise ValueError("unknown gate %r" % name)
            s.kind = GATE_KINDS[name]
            s.k = len(qubits)
            if s.k > SV_MAX_K:
                raise ValueError("gate on %d qubits (max %d)" % (s.k, SV_MAX_K))
            for j, q in enumerate(qubits):
                s.q[j] = int(q)
            for j, p in enumerate(params[:2]):
                s.params[j] = float(p)
            s.param = int(param_index)
            s.reserved = 0
            if name == "MATRIX":
                m = np.ascontiguousarray(matrix, dtype=np.complex128)
                if m.shape != (1 << s.k, 1 << s.k):
                    raise ValueError("matrix gate needs a %dx%d matrix" % (1 << s.k, 1 << s.k))
                buf = m.view(np.float64)
                self._keep.append(buf)
                s.m = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            else:
                s.m = None

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.POINTER(N.sv_gate))


def _gate_fields(g):
    """Accept objects with name/qubits/params/param_index (and .matrix for
    MATRIX gates) or tuples (name, qubits[, params[, param_index]])."""
    if isinstance(g, tuple):
        name = g[0]
        qubits = tuple(g[1])
        params = tuple(g[2]) if len(g) > 2 else ()
        pidx = g[3] if len(g) > 3 else -1
        matrix = g[4] if len(g) > 4 else None
    else:
        name, qubits = g.name, tuple(g.qubits)
        params = tuple(getattr(g, "params", ()))
        pidx = getattr(g, "param_index", -1)
        matrix = getattr(g, "matrix", None)
    name = name.upper()
    if name == "MATRIX" and matrix is None:
        raise ValueError("MATRIX gate without .matrix")
    return name, qubits, params, pidx, matrix


def gate_matrix(g) -> np.ndarray:
    """Matrix of one gate as computed by the library (host side)."""
    ga = GateArray([g])
    k = ga.arr[0].k
    out = np.zeros((1 << k) * (1 << k) * 2, dtype=np.float64)
    N.check(N.lib().sv_gate_matrix(ga.ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.view(np.complex128).reshape(1 << k, 1 << k)


def controlled(gate, controls):
    """The gate controlled by the control qubits (acting when all are 1), as a
    MATRIX gate tuple on (controls..., gate qubits) (sv_controlled_gate)."""
    ga = GateArray([gate])
    c = np.ascontiguousarray([int(x) for x in controls], dtype=np.int32)
    k = c.size + ga.arr[0].k
    m = np.zeros(2 * (1 << k) * (1 << k), dtype=np.float64)
    out = N.sv_gate()
    N.check(N.lib().sv_controlled_gate(ga.ptr, c.size, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       ctypes.byref(out), m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return ("MATRIX", tuple(int(out.q[j]) for j in range(k)), (), -1, m.view(np.complex128).reshape(1 << k, 1 << k))


def _mask(qubits) -> int:
    mask = 0
    for q in qubits:
        mask |= 1 << int(q)
    return mask


def lightcone(gates, n: int, pinned, direction: str = "right") -> List[int]:
    """Indices of the gates inside the light cone of the pinned qubits (the
    paper's pop, sv_lightcone): direction "right" walks from the end (exact for
    observables on the pinned qubits), "left" from the start."""
    ga = gates if isinstance(gates, GateArray) else GateArray(gates)
    d = {"right": N.POP_RIGHT, "left": N.POP_LEFT}.get(direction)
    if d is None:
        raise ValueError("direction must be 'right' or 'left'")
    keep = np.zeros(max(ga.n, 1), dtype=np.int32)
    cnt = ctypes.c_int()
    N.check(N.lib().sv_lightcone(ga.ptr, ga.n, int(n), _mask(pinned), d,
                                 keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(cnt)))
    return [int(x) for x in keep[:cnt.value]]


def compact_qubits(gates, n: int, pinned=()):
    """(n_used, gates, pos_map): the gates moved onto the qubits they touch
    plus the pinned ones, renumbered 0.. in ascending order
    (sv_compact_qubits); pos_map[p] is old position p's new one or -1."""
    gates = list(gates)
    ga = GateArray(gates)
    out = (N.sv_gate * max(ga.n, 1))()
    pos = np.zeros(int(n), dtype=np.int32)
    used = ctypes.c_int()
    N.check(N.lib().sv_compact_qubits(ga.ptr, ga.n, int(n), _mask(pinned), ctypes.cast(out, ctypes.POINTER(N.sv_gate)),
                                      pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(used)))
    moved = []
    for i, g in enumerate(gates):
        t = tuple(g) if isinstance(g, tuple) else (g.name, tuple(g.qubits), tuple(getattr(g, "params", ())),
                                                   getattr(g, "param_index", -1)) + (
            (g.matrix,) if getattr(g, "matrix", None) is not None else ())
        moved.append((t[0], tuple(int(out[i].q[j]) for j in range(out[i].k))) + t[2:])
    return used.value, moved, [int(x) for x in pos]


def simplify(gates, n: int, use_matrix_commutation: bool = True) -> List[int]:
    """Indices of the gates left after cancelling inverse pairs (the paper's
    simplify)."""
    ga = gates if isinstance(gates, GateArray) else GateArray(gates)
    keep = np.zeros(max(ga.n, 1), dtype=np.int32)
    cnt = ctypes.c_int()
    N.check(N.lib().sv_simplify(ga.ptr, ga.n, int(n), int(bool(use_matrix_commutation)),
                                keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(cnt)))
    return [int(x) for x in keep[:cnt.value]]


# ------------------------------------------------------------------ Pauli sums
_PAULI_BITS = {"X": (1, 0), "Y": (1, 1), "Z": (0, 1), "I": (0, 0)}


class PauliSum:
    """sv_pauli_sum from [(coef, ((position, 'X'|'Y'|'Z'), ...)), ...]."""

    def __init__(self, terms):
        terms = list(terms)
        self.coef = np.array([float(c) for c, _ in terms] or [0.0], dtype=np.float64)
        xs, zs = [], []
        for _, factors in terms:
            x = z = 0
            for q, p in factors:
                bx, bz = _PAULI_BITS[p.upper()]
                x |= bx << int(q)
                z |= bz << int(q)
            xs.append(x)
            zs.append(z)
        self.x = np.array(xs or [0], dtype=np.uint64)
        self.z = np.array(zs or [0], dtype=np.uint64)
        self.s = N.sv_pauli_sum()
        self.s.n_terms = len(terms)
        self.s.reserved = 0
        self.s.coef = self.coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.s.xmask = self.x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        self.s.zmask = self.z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))

    @property
    def ptr(self):
        return ctypes.byref(self.s)


def pauli_sum(terms) -> PauliSum:
    return PauliSum(terms)


def expectation_noalloc(tensor, n: int, terms, stream=None) -> float:
    """<psi|H|psi> of the n-qubit state held in a device tensor (complex64 as
    float32 pairs, complex128 as float64 pairs) without any device allocation
    (sv_expectation_noalloc): term tables and partials live in the library's
    fixed per-device array."""
    torch = _torch()
    dt = {torch.float32: C64, torch.float64: C128}.get(tensor.dtype)
    if dt is None or tensor.numel() < (2 << int(n)) or not tensor.is_contiguous():
        raise ValueError("expected a contiguous float32/float64 tensor of at least 2^(n+1) elements")
    H = terms if isinstance(terms, PauliSum) else PauliSum(terms)
    st = stream if stream is not None else torch.cuda.current_stream(tensor.device)
    out = ctypes.c_double()
    N.check(N.lib().sv_expectation_noalloc(ctypes.c_void_p(tensor.data_ptr()), int(n), dt,
                                           ctypes.c_void_p(st.cuda_stream), H.ptr, ctypes.byref(out)))
    return out.value


# ------------------------------------------------------------------ states
def _torch():
    import torch
    return torch


class State:
    """An n-qubit state in a torch tensor on the current HIP device.

    ``dtype`` is "c64" or "c128".  Work is enqueued on ``stream`` (default:
    torch's current stream)."""

    def __init__(self, n: int, dtype: str = "c64", stream=None, device=None):
        torch = _torch()
        self.n = int(n)
        self.dtype = C64 if dtype in ("c64", C64) else C128
        real = torch.float32 if self.dtype == C64 else torch.float64
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.tensor = torch.empty(2 << self.n, dtype=real, device=dev)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = st
        h = ctypes.c_void_p()
        N.check(N.lib().sv_alloc(self.n, self.dtype, ctypes.c_void_p(self.tensor.data_ptr()),
                                 self.tensor.numel() * self.tensor.element_size(),
                                 ctypes.c_void_p(st.cuda_stream), ctypes.byref(h)))
        self.h = h

    # -- lifetime
    def free(self):
        if getattr(self, "h", None) and self.h.value:
            N.lib().sv_free(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- contents
    def set_product(self, tokens: str):
        N.check(N.lib().sv_set_product(self.h, tokens.encode()))
        return self

    def set_basis(self, index: int):
        N.check(N.lib().sv_set_basis(self.h, int(index)))
        return self

    def read(self, first: int = 0, count: int = None) -> np.ndarray:
        count = (1 << self.n) - first if count is None else count
        out = np.empty(count, dtype=np.complex64 if self.dtype == C64 else np.complex128)
        N.check(N.lib().sv_read(self.h, int(first), int(count), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def write(self, values, first: int = 0):
        v = np.ascontiguousarray(values, dtype=np.complex64 if self.dtype == C64 else np.complex128)
        N.check(N.lib().sv_write(self.h, int(first), int(v.size), v.ctypes.data_as(ctypes.c_void_p)))
        return self

    def copy_from(self, other: "State"):
        N.check(N.lib().sv_copy(self.h, other.h))
        return self

    def synchronize(self):
        N.check(N.lib().sv_synchronize(self.h))

    # -- evolution
    def apply_gate(self, gate):
        ga = GateArray([gate])
        N.check(N.lib().sv_apply_gate(self.h, ga.ptr))
        return self

    def run(self, gates, max_k: int = SV_MAX_K, precision: int = None, rule: int = RULE_NONE,
            use_graph: bool = False, basis: int = None):
        """Fuse (rule, max_k) and apply the gates (sv_run_circuit); with
        `basis`, start from the basis state |basis> (sv_run_circuit_basis)."""
        ga = gates if isinstance(gates, GateArray) else GateArray(gates)
        o = N.sv_run_opts()
        o.max_k = int(max_k)
        o.precision = (PREC_FP32 if self.dtype == C64 else PREC_FP64) if precision is None else int(precision)
        o.rule = int(rule)
        o.use_graph = int(bool(use_graph))
        if basis is None:
            N.check(N.lib().sv_run_circuit(self.h, ga.ptr, ga.n, ctypes.byref(o)))
        else:
            N.check(N.lib().sv_run_circuit_basis(self.h, int(basis), ga.ptr, ga.n, ctypes.byref(o)))
        return self

    def apply_plan(self, plan: "Plan", precision: int = None, use_graph: bool = False):
        prec = (PREC_FP32 if self.dtype == C64 else PREC_FP64) if precision is None else int(precision)
        N.check(N.lib().sv_apply_plan(self.h, plan.h, prec, int(bool(use_graph))))
        return self

    def graph_stats(self):
        """(graph runs, runs that reused the state's instantiated graph)."""
        runs, reused = ctypes.c_int64(), ctypes.c_int64()
        N.check(N.lib().sv_graph_stats(self.h, ctypes.byref(runs), ctypes.byref(reused)))
        return runs.value, reused.value

    def stream_probe(self, tile_positions, reps: int = 10) -> float:
        """Mean ms of a streaming read + write pass over this complex64 state
        in tiles spanned by the 14 tile positions (sv_stream_probe)."""
        ms = ctypes.c_double()
        N.check(N.lib().sv_stream_probe(self.h, _mask(tile_positions), int(reps), ctypes.byref(ms)))
        return ms.value

    # -- reductions (FP64)
    def norm2(self) -> float:
        out = ctypes.c_double()
        N.check(N.lib().sv_norm(self.h, ctypes.byref(out)))
        return out.value

    def inner(self, other: "State") -> complex:
        """<self|other>."""
        re, im = ctypes.c_double(), ctypes.c_double()
        N.check(N.lib().sv_inner(self.h, other.h, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def expectation(self, terms) -> float:
        H = terms if isinstance(terms, PauliSum) else PauliSum(terms)
        out = ctypes.c_double()
        N.check(N.lib().sv_expectation(self.h, H.ptr, ctypes.byref(out)))
        return out.value

    # -- projections and measurement
    def project(self, qubits, bits: str, renormalize: bool = True) -> float:
        """psi -> |bits><bits| psi on the qubits (bits[0] on qubits[0]);
        returns ||P psi||^2 (sv_project)."""
        q = np.ascontiguousarray([int(x) for x in qubits], dtype=np.int32)
        if len(bits) != q.size or set(bits) - {"0", "1"}:
            raise ValueError("bits must be a 0/1 string with one character per qubit")
        p = ctypes.c_double()
        N.check(N.lib().sv_project(self.h, q.size, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(bits, 2),
                                   int(bool(renormalize)), ctypes.byref(p)))
        return p.value

    def measure(self, qubits, uniforms):
        """Measure the qubits one after another with the given uniforms;
        returns (bit string, probability of the outcome) (sv_measure)."""
        q = np.ascontiguousarray([int(x) for x in qubits], dtype=np.int32)
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        if u.size != q.size:
            raise ValueError("one uniform per measured qubit")
        bits, p = ctypes.c_uint64(), ctypes.c_double()
        N.check(N.lib().sv_measure(self.h, q.size, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(bits),
                                   ctypes.byref(p)))
        return format(bits.value, "0%db" % q.size), p.value

    # -- Kraus channels sampled on the state
    def kraus_probabilities(self, op: "SuperOp") -> np.ndarray:
        """||K_i psi||^2 for the Kraus operators of op (FP64 on the device)."""
        c, keep = N.sv_super_op(), []
        op.fill(c, keep)
        out = np.zeros(max(c.n_left, 1), dtype=np.float64)
        N.check(N.lib().sv_kraus_probabilities(self.h, ctypes.byref(c),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out[:c.n_left]

    def apply_kraus_sampled(self, op: "SuperOp", u: float):
        """Apply K_i / sqrt(p_i), i drawn by the uniform u; returns (i, p_i)."""
        c, keep = N.sv_super_op(), []
        op.fill(c, keep)
        i, p = ctypes.c_int32(), ctypes.c_double()
        N.check(N.lib().sv_apply_kraus_sampled(self.h, ctypes.byref(c), float(u), ctypes.byref(i), ctypes.byref(p)))
        return i.value, p.value

    def run_trajectory(self, gates, ops, uniforms, max_k: int = SV_MAX_K, precision: int = None,
                       rule: int = RULE_NONE) -> np.ndarray:
        """Gates with Kraus channels sampled among them (sv_run_trajectory);
        returns the chosen operator indices."""
        ga = gates if isinstance(gates, GateArray) else GateArray(gates)
        ops = list(ops)
        arr = (N.sv_super_op * max(len(ops), 1))()
        keep = []
        for j, op in enumerate(ops):
            op.fill(arr[j], keep)
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        if u.size != len(ops):
            raise ValueError("one uniform per operator")
        outcomes = np.zeros(max(len(ops), 1), dtype=np.int32)
        o = N.sv_run_opts()
        o.max_k = int(max_k)
        o.precision = (PREC_FP32 if self.dtype == C64 else PREC_FP64) if precision is None else int(precision)
        o.rule = int(rule)
        o.use_graph = 0
        N.check(N.lib().sv_run_trajectory(self.h, ga.ptr, ga.n, ctypes.cast(arr, ctypes.POINTER(N.sv_super_op)),
                                          len(ops), u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.byref(o), outcomes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return outcomes[:len(ops)]

    def apply_pauli_sum(self, terms, out: "State"):
        H = terms if isinstance(terms, PauliSum) else PauliSum(terms)
        N.check(N.lib().sv_apply_pauli_sum(self.h, H.ptr, out.h))
        return out


# ------------------------------------------------------------------ density matrices
class SuperOp:
    """One super operator (sv_super_op) on qubits q (q[0] the most significant
    bit of its local index), acting after the first ``after`` gates of a
    circuit.  Either a KrausSuperGate, rho -> sum_ij s[i, j] L_i rho R_j^dagger
    (``s`` None = identity: the Kraus channel when left == right), or a
    MatrixSuperGate: ``superop`` acting on the row-major vectorisation of the
    k-qubit rho (paper, Gates and Properties section)."""

    def __init__(self, qubits, left=None, right=None, s=None, superop=None, after: int = 0):
        self.qubits = tuple(int(q) for q in qubits)
        self.after = int(after)
        k = len(self.qubits)
        D = 1 << k
        as_ops = lambda ms: np.ascontiguousarray(np.array(ms, dtype=np.complex128).reshape(-1, D, D))
        self.superop = None if superop is None else np.ascontiguousarray(superop, dtype=np.complex128)
        self.left = None if left is None else as_ops(left)
        self.right = self.left if right is None else as_ops(right)
        self.s = None if s is None else np.ascontiguousarray(s, dtype=np.complex128)

    def at(self, after: int) -> "SuperOp":
        """The same operator placed after the first ``after`` gates."""
        o = SuperOp.__new__(SuperOp)
        o.__dict__.update(self.__dict__)
        o.after = int(after)
        return o

    def fill(self, c: "N.sv_super_op", keep: list):
        dp = lambda a: (keep.append(a.view(np.float64)) or keep[-1].ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        c.after = self.after
        c.k = len(self.qubits)
        if not 1 <= c.k <= 3:
            raise ValueError("super operator on %d qubits (1..3)" % c.k)
        for j, q in enumerate(self.qubits):
            c.q[j] = q
        c.reserved = 0
        if self.superop is not None:
            c.n_left = c.n_right = 0
            c.superop = dp(self.superop)
        else:
            c.n_left, c.n_right = len(self.left), len(self.right)
            c.left, c.right = dp(self.left), dp(self.right)
            if self.s is not None:
                c.s = dp(self.s)

    def matrix(self) -> np.ndarray:
        """The 4^k x 4^k matrix on the row-major vectorisation (library, host)."""
        c, keep = N.sv_super_op(), []
        self.fill(c, keep)
        D2 = 1 << (2 * len(self.qubits))
        out = np.zeros(2 * D2 * D2, dtype=np.float64)
        N.check(N.lib().sv_super_op_matrix(ctypes.byref(c), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.view(np.complex128).reshape(D2, D2)


def _super_from_c(c: "N.sv_super_op", mats: np.ndarray, s=None) -> SuperOp:
    """A SuperOp holding the operators a library constructor wrote."""
    k = c.k
    D = 1 << k
    ops = mats.view(np.complex128)[: c.n_left * D * D].reshape(c.n_left, D, D).copy()
    return SuperOp(tuple(int(c.q[j]) for j in range(k)), left=ops, s=s, after=int(c.after))


def depolarizing(qubits, p: float, after: int = 0) -> SuperOp:
    """Global depolarizing channel rho -> (1 - p) rho + p I/d on the qubits
    (paper, Noisy gates section; sv_channel_depolarizing)."""
    q = np.ascontiguousarray([int(x) for x in qubits], dtype=np.int32)
    if not 1 <= q.size <= 3:
        raise ValueError("depolarizing channel on %d qubits (1..3)" % q.size)
    mats = np.zeros(2 * 16 ** q.size, dtype=np.float64)
    c = N.sv_super_op()
    N.check(N.lib().sv_channel_depolarizing(q.size, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(p),
                                            int(after), mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            ctypes.byref(c)))
    return _super_from_c(c, mats)


_PAULI_INDEX = {"X": 1, "Y": 2, "Z": 3}


def dephasing(qubit: int, p: float, pauli: str = "Z", after: int = 0) -> SuperOp:
    """rho -> (1 - p) rho + p sigma rho sigma (paper, Noisy gates section;
    sv_channel_dephasing)."""
    if pauli.upper() not in _PAULI_INDEX:
        raise ValueError("dephasing Pauli must be X, Y or Z")
    mats = np.zeros(16, dtype=np.float64)
    c = N.sv_super_op()
    N.check(N.lib().sv_channel_dephasing(int(qubit), _PAULI_INDEX[pauli.upper()], float(p), int(after),
                                         mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(c)))
    return _super_from_c(c, mats)


def amplitude_damping(qubit: int, gamma: float, excitation: float = 0.0, after: int = 0) -> SuperOp:
    """Kraus operators sqrt(1 - excitation)|0><0| + sqrt(1 - gamma)|1><1|,
    sqrt(gamma)|0><1| and, for a nonzero excitation rate, sqrt(excitation)
    |1><0| (paper, Noisy gates section; sv_channel_amplitude_damping)."""
    mats = np.zeros(24, dtype=np.float64)
    c = N.sv_super_op()
    N.check(N.lib().sv_channel_amplitude_damping(int(qubit), float(gamma), float(excitation), int(after),
                                                 mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 ctypes.byref(c)))
    return _super_from_c(c, mats)


def pauli_channel(qubits, s, after: int = 0) -> SuperOp:
    """GlobalPauliChannel rho -> sum_ij s_ij sigma_i rho sigma_j (paper, Noisy
    gates section; sv_channel_pauli): s is 4^k x 4^k, string i = sum_j i_j
    4^(k-1-j) with i_j in 0..3 = I, X, Y, Z on qubits[j]."""
    q = np.ascontiguousarray([int(x) for x in qubits], dtype=np.int32)
    if not 1 <= q.size <= 3:
        raise ValueError("Pauli channel on %d qubits (1..3)" % q.size)
    S = np.ascontiguousarray(s, dtype=np.complex128)
    if S.shape != (4 ** q.size, 4 ** q.size):
        raise ValueError("s must be %dx%d" % (4 ** q.size, 4 ** q.size))
    mats = np.zeros(2 * 16 ** q.size, dtype=np.float64)
    c = N.sv_super_op()
    N.check(N.lib().sv_channel_pauli(q.size, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     S.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     int(after), mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     ctypes.byref(c)))
    return _super_from_c(c, mats, s=S)


def local_channels(make, qubits, *params, after: int = 0) -> List[SuperOp]:
    """The paper's Local version of a one-qubit channel: make(qubit, *params)
    on each qubit, each parameter either one value for every qubit or one
    value per qubit."""
    qubits = list(qubits)
    cols = []
    for v in params:
        seq = list(v) if isinstance(v, (list, tuple, np.ndarray)) and np.ndim(v) == 1 and len(v) == len(qubits) \
            and not isinstance(v, str) else [v] * len(qubits)
        cols.append(seq)
    return [make(q, *[c[i] for c in cols], after=after) for i, q in enumerate(qubits)]


def kraus_form(op: SuperOp) -> SuperOp:
    """The Kraus form of a KrausSuperGate with right == left and Hermitian
    PSD s (sv_kraus_form)."""
    c, keep = N.sv_super_op(), []
    op.fill(c, keep)
    mats = np.zeros(2 * max(c.n_left, 1) * (1 << (2 * c.k)), dtype=np.float64)
    out = N.sv_super_op()
    N.check(N.lib().sv_kraus_form(ctypes.byref(c), mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(out)))
    return _super_from_c(out, mats)


class DensityMatrix:
    """Density matrix of n qubits held row-major in a State of 2n qubits
    (rho[r][c] at amplitude r 2^n + c); starts as |0..0><0..0|."""

    def __init__(self, n: int, dtype: str = "c64", stream=None, device=None):
        self.n = int(n)
        self.state = State(2 * self.n, dtype, stream, device).set_basis(0)

    @property
    def dtype(self):
        return self.state.dtype

    def set_basis(self, index: int):
        """|index><index|."""
        self.state.set_basis((int(index) << self.n) | int(index))
        return self

    def run(self, gates, ops=(), max_k: int = SV_MAX_K, precision: int = None, rule: int = RULE_NONE,
            use_graph: bool = False):
        """Evolve by the gates with the super operators among them (sv_dm_run)."""
        ga = gates if isinstance(gates, GateArray) else GateArray(gates)
        ops = list(ops)
        arr = (N.sv_super_op * max(len(ops), 1))()
        keep = []
        for j, op in enumerate(ops):
            op.fill(arr[j], keep)
        o = N.sv_run_opts()
        o.max_k = int(max_k)
        o.precision = (PREC_FP32 if self.dtype == C64 else PREC_FP64) if precision is None else int(precision)
        o.rule = int(rule)
        o.use_graph = int(bool(use_graph))
        N.check(N.lib().sv_dm_run(self.state.h, ga.ptr, ga.n, ctypes.cast(arr, ctypes.POINTER(N.sv_super_op)),
                                  len(ops), ctypes.byref(o)))
        return self

    def expectation(self, terms) -> float:
        """Tr(rho H) in FP64 on the device."""
        H = terms if isinstance(terms, PauliSum) else PauliSum(terms)
        out = ctypes.c_double()
        N.check(N.lib().sv_dm_expectation(self.state.h, H.ptr, ctypes.byref(out)))
        return out.value

    def trace(self) -> float:
        return self.expectation([(1.0, ())])

    def read(self) -> np.ndarray:
        """rho as a 2^n x 2^n array (reads all 4^n entries)."""
        d = 1 << self.n
        return self.state.read().reshape(d, d)


def fidelity_error(ref: State, psi: State) -> float:
    """1 - |<ref|psi>|^2 / (||ref||^2 ||psi||^2), all in FP64 on the device."""
    ov = ref.inner(psi)
    return 1.0 - abs(ov) ** 2 / (ref.norm2() * psi.norm2())


# ------------------------------------------------------------------ fusion
@dataclass
class Block:
    qubits: tuple
    members: list
    matrix: np.ndarray
    tile_pass: int = -1


class Plan:
    """A fused plan (sv_fuse, or sv_fuse_prec for a given precision); blocks
    are read back on demand."""

    def __init__(self, gates, n: int, max_k: int, rule: int = RULE_PAPER, precision: int = None):
        ga = gates if isinstance(gates, GateArray) else GateArray(gates)
        h = ctypes.c_void_p()
        if precision is None:
            N.check(N.lib().sv_fuse(ga.ptr, ga.n, int(n), int(max_k), int(rule), ctypes.byref(h)))
        else:
            N.check(N.lib().sv_fuse_prec(ga.ptr, ga.n, int(n), int(max_k), int(rule), int(precision),
                                         ctypes.byref(h)))
        self.h = h
        self.n = n

    def __del__(self):
        try:
            if self.h and self.h.value:
                N.lib().sv_plan_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    @property
    def rule(self) -> int:
        out = ctypes.c_int()
        N.check(N.lib().sv_plan_rule(self.h, ctypes.byref(out)))
        return out.value

    @property
    def max_k(self) -> int:
        out = ctypes.c_int()
        N.check(N.lib().sv_plan_max_k(self.h, ctypes.byref(out)))
        return out.value

    def __len__(self) -> int:
        out = ctypes.c_int()
        N.check(N.lib().sv_plan_num_blocks(self.h, ctypes.byref(out)))
        return out.value

    def block(self, b: int, with_matrix: bool = True) -> Block:
        k = ctypes.c_int32()
        q = (ctypes.c_int32 * SV_MAX_K)()
        nm = ctypes.c_int32()
        N.check(N.lib().sv_plan_block(self.h, b, ctypes.byref(k), q, ctypes.byref(nm)))
        members = (ctypes.c_int32 * max(nm.value, 1))()
        N.check(N.lib().sv_plan_block_members(self.h, b, members))
        mat = None
        if with_matrix:
            D = 1 << k.value
            buf = np.zeros(2 * D * D, dtype=np.float64)
            N.check(N.lib().sv_plan_block_matrix(self.h, b, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
            mat = buf.view(np.complex128).reshape(D, D)
        tp = ctypes.c_int32()
        N.check(N.lib().sv_plan_block_pass(self.h, b, ctypes.byref(tp)))
        return Block(tuple(q[:k.value]), list(members[:nm.value]), mat, tp.value)

    def blocks(self, with_matrix: bool = True) -> List[Block]:
        return [self.block(b, with_matrix) for b in range(len(self))]


def fuse(gates, n: int, max_k: int, rule: int = RULE_PAPER, precision: int = None) -> Plan:
    return Plan(gates, n, max_k, rule, precision)


# ------------------------------------------------------------------ gradients
def backward(psi: State, scratch: State, gates, terms, n_params: int, precision: int = None) -> np.ndarray:
    """Adjoint dE/dtheta (sv_backward, or sv_backward_prec with a
    precision); psi holds the forward output and is consumed."""
    ga = gates if isinstance(gates, GateArray) else GateArray(gates)
    H = terms if isinstance(terms, PauliSum) else PauliSum(terms)
    grad = np.zeros(max(int(n_params), 1), dtype=np.float64)
    gp = grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if precision is None:
        N.check(N.lib().sv_backward(psi.h, scratch.h, ga.ptr, ga.n, H.ptr, gp, int(n_params)))
    else:
        N.check(N.lib().sv_backward_prec(psi.h, scratch.h, ga.ptr, ga.n, H.ptr, gp, int(n_params), int(precision)))
    return grad[:n_params]


def _bind_thetas(gates, thetas):
    out = []
    for g in gates:
        name, qubits, params, pidx, matrix = _gate_fields(g)
        if pidx >= 0:
            params = (float(thetas[pidx]),) + tuple(params[1:])
        out.append((name, qubits, params, pidx, matrix))
    return out


def _energy_function():
    torch = _torch()

    class Energy(torch.autograd.Function):
        """E(theta) = <psi(theta)|H|psi(theta)> with the adjoint backward.

        forward(thetas, n, gates, terms, max_k, precision): gates carry
        param_index >= 0 on differentiable rotations; thetas is a CPU or CUDA
        float64 tensor.  The forward state is kept for the backward pass,
        which consumes it (two state buffers, no stored trajectory)."""

        @staticmethod
        def forward(ctx, thetas, n, gates, terms, max_k=SV_MAX_K, rule=RULE_PAPER):
            th = thetas.detach().double().cpu().numpy()
            bound = _bind_thetas(gates, th)
            psi = State(n, "c64")
            psi.run(bound, max_k=max_k, rule=rule)
            H = PauliSum(terms)
            e = psi.expectation(H)
            ctx.save = (psi, bound, H, n, th.size)
            return thetas.new_tensor(e)

        @staticmethod
        def backward(ctx, grad_out):
            psi, bound, H, n, npar = ctx.save
            scratch = State(n, "c64")
            g = backward(psi, scratch, bound, H, npar)
            ctx.save = None
            gt = torch.as_tensor(g, dtype=torch.float64, device=grad_out.device) * grad_out
            return gt, None, None, None, None, None

    return Energy


class _EnergyProxy:
    _fn = None

    def apply(self, *args):
        if _EnergyProxy._fn is None:
            _EnergyProxy._fn = _energy_function()
        return _EnergyProxy._fn.apply(*args)


Energy = _EnergyProxy()


# ------------------------------------------------------------------ batches
class Batch:
    """Many trajectories of different qubit counts run together
    (sv_batch_create / sv_batch_run)."""

    def __init__(self, circuits, max_k: int = -1, stream=None, precision: int = PREC_FP32):
        """precision: PREC_FP32, PREC_SPLIT_BF16, PREC_SPLIT_FP16 or PREC_SPLIT_BF16X3 for the
        tile passes of the trajectories with 14 or more qubits."""
        torch = _torch()
        circuits = list(circuits)
        self.n_qubits = np.array([int(n) for n, _ in circuits], dtype=np.int32)
        offs = [0]
        flat = []
        for _, gates in circuits:
            flat.extend(gates)
            offs.append(len(flat))
        self.offsets = np.array(offs, dtype=np.int64)
        self.gates = GateArray(flat)
        d = N.sv_batch_desc()
        d.n_traj = len(circuits)
        d.max_k = int(max_k)
        d.n_qubits = self.n_qubits.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.gate_offsets = self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.gates = self.gates.ptr
        d.precision = int(precision)
        self.desc = d
        need = ctypes.c_size_t()
        N.check(N.lib().sv_batch_required_bytes(ctypes.byref(d), ctypes.byref(need)))
        self.tensor = torch.empty(max(need.value // 4, 1), dtype=torch.float32, device="cuda")
        st = stream if stream is not None else torch.cuda.current_stream()
        self.stream = st
        h = ctypes.c_void_p()
        N.check(N.lib().sv_batch_create(ctypes.byref(d), ctypes.c_void_p(self.tensor.data_ptr()),
                                        self.tensor.numel() * 4, ctypes.c_void_p(st.cuda_stream),
                                        ctypes.byref(h)))
        self.h = h

    def run(self, use_graph: bool = True) -> np.ndarray:
        z = np.zeros(len(self.n_qubits), dtype=np.float64)
        N.check(N.lib().sv_batch_run(self.h, int(bool(use_graph)), z.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return z

    def read(self, t: int, first: int = 0, count: int = None) -> np.ndarray:
        n = int(self.n_qubits[t])
        count = (1 << n) - first if count is None else count
        out = np.empty(count, dtype=np.complex64)
        N.check(N.lib().sv_batch_read(self.h, int(t), int(first), int(count), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def __del__(self):
        try:
            if self.h and self.h.value:
                N.lib().sv_batch_free(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass


# ------------------------------------------------------------------ tuning / stats
def autotune(scratch: State, precision: int = PREC_FP32) -> np.ndarray:
    cost = np.zeros(SV_MAX_K + 1, dtype=np.float64)
    N.check(N.lib().sv_autotune(scratch.h, int(precision), cost.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return cost


def set_cost_table(n: int, precision: int, cost) -> None:
    c = np.ascontiguousarray(cost, dtype=np.float64)
    assert c.size == SV_MAX_K + 1
    N.check(N.lib().sv_set_cost_table(int(n), int(precision), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def tune_cache_load(path: str = None) -> int:
    """Install the cost tables and launch shapes saved in a tuning cache
    (sv_tune_cache_load; path None = $SV_TUNE_CACHE); returns the count."""
    n = ctypes.c_int()
    N.check(N.lib().sv_tune_cache_load(None if path is None else path.encode(), ctypes.byref(n)))
    return n.value


TILE_SHAPES = ((14, 8), (14, 16), (13, 4), (13, 8))
MAX_TILE_LAUNCH_BLOCKS = 16  # blocks one tile-pass launch can hold (stats classes k = 1..16)


def set_tile_shape(tile_bits: int, waves: int) -> None:
    """Launch shape of the tile passes: 2^tile_bits amplitudes per LDS tile,
    `waves` waves per workgroup (one of TILE_SHAPES), for the whole process."""
    N.check(N.lib().sv_set_tile_shape(int(tile_bits), int(waves)))


def get_tile_shape():
    """(tile_bits, waves, blocks per launch) of the tile passes (sv_get_tile_shape)."""
    b, w, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    N.check(N.lib().sv_get_tile_shape(ctypes.byref(b), ctypes.byref(w), ctypes.byref(m)))
    return b.value, w.value, m.value


def tile_placement(blocks, n: int, tile_bits: int = 14, waves: int = 16, precision: int = PREC_SPLIT_BF16):
    """Layout of one tile pass of 4-qubit blocks (sv_tile_placement): the
    state position of each tile bit, the LDS image of each tile bit, and the
    extra LDS cycles the model counts for that placement."""
    pos = np.ascontiguousarray([sorted(int(q) for q in b) for b in blocks], dtype=np.int32).reshape(-1)
    tp = np.zeros(tile_bits, dtype=np.int32)
    img = np.zeros(tile_bits, dtype=np.uint32)
    c = ctypes.c_int32()
    N.check(N.lib().sv_tile_placement(len(blocks), pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(n),
                                      int(tile_bits), int(waves), int(precision),
                                      tp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      img.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(c)))
    return tp, img, c.value


def set_tile_union(max_positions: int) -> None:
    """Position limit (8..10) of the passes the tiled rule plans."""
    N.check(N.lib().sv_set_tile_union(int(max_positions)))


def stats_enable(on: bool = True) -> None:
    N.check(N.lib().sv_stats_enable(int(bool(on))))


def stats_reset() -> None:
    N.check(N.lib().sv_stats_reset())


FAMILIES = {"reg": 1, "generic": 2, "mfma_f32": 3, "split_bf16": 4, "split_fp16": 5,
            "reduce": 6, "adjoint": 7, "batch": 8, "tile": 9, "tile_bf16": 10, "tile_fp16": 11, "tile_bf16x3": 12}


def stats_query(family: str, k: int):
    """(launch count, summed device milliseconds) of a kernel class."""
    cls = 100 * FAMILIES[family] + int(k)
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    N.check(N.lib().sv_stats_query(cls, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value
