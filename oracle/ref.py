"""Oracle: plain complex128 state-vector evolution -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never does.  It shares no code with the HIP library.

Every function follows the plain definition of what the paper's state-vector
method computes (Simulations / State Vector sections): the output state is the
ordered product of the circuit's gates applied to the initial state.  Pins that
tie each function to the paper or to mathematics live in tests/test_oracle_pins.py.

Conventions
-----------
* Bit order: amplitude index i holds the qubit at position p in bit p.  The
  paper's arrays are ``(2,)*n`` with axis j following ``order[j]`` in C order,
  so ``order[0]`` is the most significant bit (the Grover worked example prints
  its negative amplitudes at 000 and 100, which fixes this).
* A k-qubit matrix's local index m has its most significant bit on qubits[0].
* Rotations: R_P(theta) = exp(-i theta P / 2)  (a reading; the paper only fixes
  R(theta)**p = R(p theta) in the Gates and Properties section).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_ref.c")
_LIB_PATH = os.path.join(_HERE, "libsvref.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile sv_ref.c with gcc (OpenMP over independent amplitude groups)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.ref_product_state.argtypes = [ctypes.c_int, ctypes.c_char_p, dp]
        L.ref_product_state.restype = ctypes.c_int
        L.ref_apply.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp]
        L.ref_apply.restype = None
        L.ref_run.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip,
                              ctypes.POINTER(ctypes.c_int64), dp, ctypes.POINTER(ctypes.c_int64)]
        L.ref_run.restype = None
        L.ref_inner.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.ref_inner.restype = None
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# --------------------------------------------------------------------------
# O4: gate table (FP64).  Gates and Properties section names the gates (H, X,
# RX, CPHASE, CX, ISWAP, FSIM, ...) but prints no matrices; these are the
# textbook definitions under the readings stated in the module docstring.
# --------------------------------------------------------------------------
_I2 = np.eye(2, dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)
_H = np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2)
_W = (_X + _Y) / math.sqrt(2)
PAULI = {"I": _I2, "X": _X, "Y": _Y, "Z": _Z}


def _principal_sqrt_of_pauli_like(P: np.ndarray) -> np.ndarray:
    # For P with P^2 = I and eigenvalues +-1, the principal square root is
    # ((1+i) I + (1-i) P) / 2 (eigenvalue 1 -> 1, eigenvalue -1 -> i).
    return ((1 + 1j) * _I2 + (1 - 1j) * P) / 2


def _rotation(P: np.ndarray, theta: float) -> np.ndarray:
    return math.cos(theta / 2) * _I2 - 1j * math.sin(theta / 2) * P


def gate_matrix(name: str, params: Sequence[float] = ()) -> np.ndarray:
    """Matrix of a named gate; for two-qubit gates the first qubit is the
    most significant bit of the 4x4 local index."""
    name = name.upper()
    if name in PAULI:
        return PAULI[name].copy()
    if name == "H":
        return _H.copy()
    if name == "SQRT_X":
        return _principal_sqrt_of_pauli_like(_X)
    if name == "SQRT_Y":
        return _principal_sqrt_of_pauli_like(_Y)
    if name == "SQRT_W":
        return _principal_sqrt_of_pauli_like(_W)
    if name in ("RX", "RY", "RZ"):
        return _rotation({"RX": _X, "RY": _Y, "RZ": _Z}[name], float(params[0]))
    if name == "CZ":
        return np.diag([1, 1, 1, -1]).astype(complex)
    if name == "CPHASE":
        return np.diag([1, 1, 1, np.exp(1j * float(params[0]))])
    if name == "CX":
        # control on the first qubit (most significant local bit)
        return np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    if name == "SWAP":
        return np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=complex)
    if name == "FSIM":
        th, ph = float(params[0]), float(params[1])
        c, s = math.cos(th), math.sin(th)
        return np.array([[1, 0, 0, 0],
                         [0, c, -1j * s, 0],
                         [0, -1j * s, c, 0],
                         [0, 0, 0, np.exp(-1j * ph)]], dtype=complex)
    raise ValueError("unknown gate %r" % name)


ROTATION_GENERATOR = {"RX": "X", "RY": "Y", "RZ": "Z"}


def matrix_of(g) -> np.ndarray:
    """Matrix of a workloads.Gate.  'MATRIX' gates take their matrix from the
    input generator (it is an input, drawn from a seed)."""
    if g.name == "MATRIX":
        from workloads.circuits import haar_unitary_from_seed
        return haar_unitary_from_seed(int(g.params[0]), len(g.qubits))
    return gate_matrix(g.name, g.params)


# --------------------------------------------------------------------------
# O2 / O3 / O5: product states, gate application, circuits
# --------------------------------------------------------------------------
def product_state(n: int, tokens: str) -> np.ndarray:
    """Initial and Final State Specification section: tokens 0 1 + -; a single
    character is broadcast to all n qubits."""
    if len(tokens) == 1:
        tokens = tokens * n
    if len(tokens) != n:
        raise ValueError("need n tokens")
    psi = np.empty(1 << n, dtype=np.complex128)
    rc = lib().ref_product_state(n, tokens.encode(), _dptr(psi))
    if rc != 0:
        raise ValueError("bad token in %r" % tokens)
    return psi


def basis_state(n: int, index: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[index] = 1.0
    return psi


def apply(psi: np.ndarray, M: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """O3 in place on ``psi`` (complex128, length 2^n)."""
    n = int(psi.size).bit_length() - 1
    k = len(qubits)
    M = np.ascontiguousarray(M, dtype=np.complex128)
    assert M.shape == (1 << k, 1 << k)
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    assert len(set(qubits)) == k and all(0 <= x < n for x in qubits)
    lib().ref_apply(n, _dptr(psi), k, _iptr(q), _dptr(M))
    return psi


def run_matrices(psi: np.ndarray, ops: Sequence[Tuple[np.ndarray, Sequence[int]]]) -> np.ndarray:
    """O5: apply (matrix, qubits) pairs in list order, in place."""
    n = int(psi.size).bit_length() - 1
    if not ops:
        return psi
    ks = np.array([len(q) for _, q in ops], dtype=np.int32)
    for _, q in ops:
        assert len(set(q)) == len(q) and all(0 <= x < n for x in q)
    qs = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.int32) for _, q in ops]))
    qoff = np.zeros(len(ops), dtype=np.int64)
    qoff[1:] = np.cumsum(ks)[:-1]
    mats = [np.ascontiguousarray(M, dtype=np.complex128).ravel() for M, _ in ops]
    moff = np.zeros(len(ops), dtype=np.int64)
    moff[1:] = 2 * np.cumsum([m.size for m in mats])[:-1]
    ms = np.ascontiguousarray(np.concatenate(mats)).view(np.float64)
    lib().ref_run(n, _dptr(psi), len(ops), _iptr(ks), _iptr(qs),
                  qoff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(ms),
                  moff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return psi


def simulate(n: int, gates, initial: str = "0", psi: np.ndarray = None) -> np.ndarray:
    """Apply a list of workloads.Gate to a product state (or to ``psi``)."""
    if psi is None:
        psi = product_state(n, initial)
    return run_matrices(psi, [(matrix_of(g), g.qubits) for g in gates])


def inverse_ops(gates) -> List[Tuple[np.ndarray, Tuple[int, ...]]]:
    """Circuit inverse (the paper's Circuit utilities example inverts a circuit):
    reversed order, each matrix replaced by its conjugate transpose."""
    return [(matrix_of(g).conj().T, g.qubits) for g in reversed(list(gates))]


# --------------------------------------------------------------------------
# O6: metrics (FP64)
# --------------------------------------------------------------------------
def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a|b>, compensated summation in index order."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    n = int(a.size).bit_length() - 1
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().ref_inner(n, _dptr(a), _dptr(b), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def norm2(psi: np.ndarray) -> float:
    return inner(psi, psi).real


def fidelity_error(ref: np.ndarray, psi: np.ndarray) -> float:
    """1 - |<ref|psi>|^2 / (||ref||^2 ||psi||^2): blind to a global phase and
    to the norms of both states."""
    ov = inner(ref, psi.astype(np.complex128))
    return 1.0 - abs(ov) ** 2 / (norm2(ref) * norm2(psi.astype(np.complex128)))


def fidelity_error_raw(ref: np.ndarray, psi: np.ndarray) -> float:
    """|1 - |<ref|psi>|^2 / ||ref||^2| with psi NOT renormalised: the reference
    (an exact evolution of a unit state) is taken as the unit vector, so a norm
    error of psi shows up here while fidelity_error hides it."""
    ov = inner(ref, psi.astype(np.complex128))
    return abs(1.0 - abs(ov) ** 2 / norm2(ref))


def max_abs(ref: np.ndarray, psi: np.ndarray) -> float:
    """max_i |ref_i - psi_i| (complex modulus, no phase alignment)."""
    return float(np.max(np.abs(ref - psi.astype(np.complex128))))


# --------------------------------------------------------------------------
# O7: Pauli-sum expectation.  E = sum_t c_t Re <psi| P_t psi>, where P_t psi is
# built by applying each single-qubit Pauli factor with O3 on a copy.
# --------------------------------------------------------------------------
def pauli_apply(psi: np.ndarray, factors) -> np.ndarray:
    out = psi.copy()
    for (q, p) in factors:
        apply(out, PAULI[p], (q,))
    return out


def expectation(psi: np.ndarray, terms) -> float:
    e = 0.0
    for (c, factors) in terms:
        e += c * inner(psi, pauli_apply(psi, factors)).real
    return e


# --------------------------------------------------------------------------
# O8: gradients of E(theta) = <psi(theta)|H|psi(theta)> for circuits whose
# rotations R_P(theta) = exp(-i theta P/2) each use their own parameter.
# Parameter shift: dE/dtheta = [E(theta + pi/2) - E(theta - pi/2)] / 2 (exact
# for such rotations).  Central differences with step h.
# --------------------------------------------------------------------------
def energy(n: int, gates, thetas, terms, initial: str = "0") -> float:
    from workloads.circuits import with_thetas
    psi = simulate(n, with_thetas(gates, thetas), initial)
    return expectation(psi, terms)


def param_shift_grad(n, gates, thetas, terms, indices=None, initial="0") -> np.ndarray:
    thetas = np.asarray(thetas, dtype=np.float64)
    idx = range(len(thetas)) if indices is None else indices
    out = []
    for p in idx:
        tp = thetas.copy(); tp[p] += math.pi / 2
        tm = thetas.copy(); tm[p] -= math.pi / 2
        out.append(0.5 * (energy(n, gates, tp, terms, initial) - energy(n, gates, tm, terms, initial)))
    return np.array(out)


def fd_grad(n, gates, thetas, terms, h=1e-3, indices=None, initial="0") -> np.ndarray:
    thetas = np.asarray(thetas, dtype=np.float64)
    idx = range(len(thetas)) if indices is None else indices
    out = []
    for p in idx:
        tp = thetas.copy(); tp[p] += h
        tm = thetas.copy(); tm[p] -= h
        out.append((energy(n, gates, tp, terms, initial) - energy(n, gates, tm, terms, initial)) / (2 * h))
    return np.array(out)


# --------------------------------------------------------------------------
# O9: the paper's greedy fusion rule (Circuit utilities section, compress).
# For each gate in order, find the last block that shares a qubit with it;
# merge the gate into that block when the union has at most max_k qubits,
# otherwise (or when no block shares a qubit) open a new block.  Block qubits
# are listed in ascending order.  Merging into the last intersecting block is
# legal because every later block is disjoint from the gate, so the gate
# commutes past them.
# --------------------------------------------------------------------------
def fuse_paper(qubit_lists: Sequence[Sequence[int]], max_k: int):
    blocks: List[Dict] = []
    for gi, qs in enumerate(qubit_lists):
        qs = set(qs)
        target = None
        for b in reversed(blocks):
            if b["qubits"] & qs:
                target = b
                break
        if target is not None and len(target["qubits"] | qs) <= max_k:
            target["qubits"] |= qs
            target["members"].append(gi)
        else:
            blocks.append({"qubits": set(qs), "members": [gi]})
    return [(tuple(sorted(b["qubits"])), list(b["members"])) for b in blocks]


def block_matrix(ops: Sequence[Tuple[np.ndarray, Sequence[int]]], block_qubits: Sequence[int]) -> np.ndarray:
    """Matrix of an ordered list of (matrix, qubits) acting inside
    ``block_qubits`` (listed so that block_qubits[0] is the most significant
    local bit): column c is the k-qubit state |c> evolved by O3."""
    k = len(block_qubits)
    D = 1 << k
    local = {q: k - 1 - j for j, q in enumerate(block_qubits)}
    U = np.zeros((D, D), dtype=np.complex128)
    for c in range(D):
        col = basis_state(k, c)
        for M, qs in ops:
            apply(col, M, [local[q] for q in qs])
        U[:, c] = col
    return U


# --------------------------------------------------------------------------
# O10: trajectories.  The inserted Paulis are already in each trajectory's
# gate list (drawn by the input generator); the oracle just evolves it and
# reports <Z_0>.
# --------------------------------------------------------------------------
def z0(psi: np.ndarray) -> float:
    return expectation(psi, [(1.0, ((0, "Z"),))])


def trajectory_z0(traj) -> float:
    return z0(simulate(traj.n, traj.gates, "0"))
