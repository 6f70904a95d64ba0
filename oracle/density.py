"""Oracle: plain complex128 density-matrix evolution -- TEST INFRASTRUCTURE ONLY.

Only tests use this module; the product path never does.  It shares no code
with the HIP library.

What it computes (paper, Gates and Properties section: KrausSuperGate
rho -> sum_ij s_ij L_i rho R_j^dagger and MatrixSuperGate, a matrix acting on
the vectorised rho; Noisy gates section: the depolarizing, dephasing and
amplitude-damping channels; Simulations section: density matrices evolve by the
same gates as states, rho -> U rho U^dagger):

* rho is a 2^n x 2^n complex128 array, rho[r][c], with the state-vector bit
  order of ``ref`` on both indices.
* A gate or left operator acts on rho's columns with ``ref.apply``; a right
  operator R enters as (R A^dagger)^dagger.  No vectorisation is used except
  for a MatrixSuperGate, whose matrix is defined on one: the row-major
  vectorisation v[r 2^n + c] = rho[r][c] (that of kron(psi, conj(psi)) in the
  paper's State Vector example), applied with ``ref.apply`` as a gate on the
  2k positions (q + n, q), row bits most significant.

Pins: tests/test_oracle_density.py (closed forms of the channels, pure
circuits against psi psi^dagger, exact enumeration of sampled Pauli errors,
trace / Hermiticity / positivity).
"""
from __future__ import annotations

import itertools
from typing import Sequence

import numpy as np

from . import ref

PAULI = {"I": np.eye(2, dtype=np.complex128),
         "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
         "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128)}


def zero(n: int) -> np.ndarray:
    """|0..0><0..0|."""
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[0, 0] = 1.0
    return rho


def pure(psi: np.ndarray) -> np.ndarray:
    """psi psi^dagger."""
    return np.outer(psi, psi.conj())


def _left(rho: np.ndarray, M: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """M rho: M applied to every column."""
    out = np.empty_like(rho)
    for c in range(rho.shape[1]):
        col = np.ascontiguousarray(rho[:, c])
        out[:, c] = ref.apply(col, M, qubits)
    return out


def apply_gate(rho: np.ndarray, U: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """U rho U^dagger = (U (U rho)^dagger)^dagger."""
    A = _left(rho, U, qubits)
    return _left(A.conj().T.copy(), U, qubits).conj().T.copy()


def apply_kraus_super(rho: np.ndarray, left, right, s, qubits: Sequence[int]) -> np.ndarray:
    """sum_ij s[i][j] L_i rho R_j^dagger; s None = identity."""
    out = np.zeros_like(rho)
    for i, L in enumerate(left):
        A = _left(rho, L, qubits)          # L_i rho
        Ad = A.conj().T.copy()
        for j, R in enumerate(right):
            w = (1.0 if i == j else 0.0) if s is None else s[i][j]
            if w == 0:
                continue
            out += w * _left(Ad, R, qubits).conj().T  # (R_j (L_i rho)^dagger)^dagger
    return out


def apply_matrix_super(rho: np.ndarray, S: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """A MatrixSuperGate: S on the row-major vectorisation of the k-qubit rho."""
    n = rho.shape[0].bit_length() - 1
    v = rho.ravel().copy()  # v[r 2^n + c] = rho[r][c]
    pos = [q + n for q in qubits] + list(qubits)
    ref.apply(v, S, pos)
    return v.reshape(rho.shape)


def apply_op(rho: np.ndarray, op: dict) -> np.ndarray:
    """op: {"qubits", and "superop" or "left" (+ optional "right", "s")}."""
    if op.get("superop") is not None:
        return apply_matrix_super(rho, op["superop"], op["qubits"])
    left = op["left"]
    right = op.get("right") if op.get("right") is not None else left
    return apply_kraus_super(rho, left, right, op.get("s"), op["qubits"])


def simulate(n: int, gates, ops=(), rho: np.ndarray = None) -> np.ndarray:
    """Gates (workloads.Gate) in order, each op dict applied after the first
    op["after"] gates (ops in list order)."""
    rho = zero(n) if rho is None else rho.copy()
    ops = list(ops)
    j = 0
    for i, g in enumerate(list(gates) + [None]):
        while j < len(ops) and ops[j]["after"] <= i:
            rho = apply_op(rho, ops[j])
            j += 1
        if g is None:
            break
        rho = apply_gate(rho, ref.matrix_of(g), g.qubits)
    assert j == len(ops), "an op's 'after' exceeds the gate count"
    return rho


def expectation(rho: np.ndarray, terms) -> float:
    """sum_t c_t Re Tr(P_t rho), P_t rho built column by column."""
    e = 0.0
    for c, factors in terms:
        A = rho.copy()
        for q, p in factors:
            A = _left(A, PAULI[p], (q,))
        e += c * np.trace(A).real
    return e


# -------------------------------------------------------------- channels
# Kraus operators of the Noisy gates section's channels, written from their
# definitions.  Multi-qubit Pauli strings put the first label on the most
# significant local bit.
def pauli_string(labels: str) -> np.ndarray:
    m = np.ones((1, 1), dtype=np.complex128)
    for c in labels:
        m = np.kron(m, PAULI[c])
    return m


def depolarizing(qubits, p: float, after: int = 0) -> dict:
    """rho -> (1 - p) rho + p I/d: Kraus operators sqrt(1 - p + p/d^2) I and
    sqrt(p/d^2) P for the other d^2 - 1 Pauli strings P."""
    k = len(qubits)
    d = 1 << k
    ops = []
    for labels in itertools.product("IXYZ", repeat=k):
        w = p / (d * d) + (1.0 - p if set(labels) == {"I"} else 0.0)
        ops.append(np.sqrt(w) * pauli_string("".join(labels)))
    return {"qubits": tuple(qubits), "left": ops, "after": after}


def dephasing(qubit: int, p: float, pauli: str = "Z", after: int = 0) -> dict:
    """rho -> (1 - p) rho + p sigma rho sigma."""
    return {"qubits": (qubit,), "left": [np.sqrt(1 - p) * PAULI["I"], np.sqrt(p) * PAULI[pauli]], "after": after}


def amplitude_damping(qubit: int, gamma: float, excitation: float = 0.0, after: int = 0) -> dict:
    """Kraus operators sqrt(1 - excitation)|0><0| + sqrt(1 - gamma)|1><1| and
    sqrt(gamma)|0><1|, plus sqrt(excitation)|1><0| for a nonzero excitation
    rate (the generalized channel: |1> -> |0> with probability gamma, |0> ->
    |1> with probability excitation).  excitation = 0 is the paper's pair."""
    K0 = np.array([[np.sqrt(1 - excitation), 0], [0, np.sqrt(1 - gamma)]], dtype=np.complex128)
    K1 = np.array([[0, np.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    ops = [K0, K1]
    if excitation > 0:
        ops.append(np.array([[0, 0], [np.sqrt(excitation), 0]], dtype=np.complex128))
    return {"qubits": (qubit,), "left": ops, "after": after}


def pauli_channel(qubits, s, after: int = 0) -> dict:
    """GlobalPauliChannel rho -> sum_ij s_ij sigma_i rho sigma_j over the 4^k
    Pauli strings; string i has base-4 digits (first digit on qubits[0]) 0..3
    = I, X, Y, Z.  A KrausSuperGate with left = right = the strings."""
    k = len(qubits)
    strings = [pauli_string("".join(t)) for t in itertools.product("IXYZ", repeat=k)]
    return {"qubits": tuple(qubits), "left": strings, "s": np.asarray(s, dtype=np.complex128), "after": after}


# -------------------------------------------------------------- sampling on pure states
# Simulations with noise section: a channel sum_i K_i rho K_i^dagger can be
# sampled on a pure state.  Outcome i has weight p_i = ||K_i psi||^2; the
# uniform u picks the first i with a nonzero weight whose running sum exceeds
# u * sum(p), and psi becomes K_i psi / sqrt(p_i).
def kraus_probabilities(psi: np.ndarray, kraus, qubits: Sequence[int]):
    return [ref.norm2(ref.apply(psi.copy(), K, qubits)) for K in kraus]


def sample_kraus(psi: np.ndarray, kraus, qubits: Sequence[int], u: float):
    p = kraus_probabilities(psi, kraus, qubits)
    total = sum(p)
    pick, run = -1, 0.0
    for i, w in enumerate(p):
        run += w
        if w > 0:
            pick = i
            if u * total < run:
                break
    out = ref.apply(psi.copy(), kraus[pick], qubits) / np.sqrt(p[pick])
    return out, pick


def trajectory(n: int, gates, ops, uniforms, initial: str = "0"):
    """Gates in order with the Kraus channels ops (dicts with "left",
    "qubits", "after") sampled by uniforms[j]; returns (psi, outcomes)."""
    psi = ref.product_state(n, initial)
    ops = list(ops)
    outcomes = []
    j = 0
    for i, g in enumerate(list(gates) + [None]):
        while j < len(ops) and ops[j]["after"] <= i:
            psi, pick = sample_kraus(psi, ops[j]["left"], ops[j]["qubits"], uniforms[j])
            outcomes.append(pick)
            j += 1
        if g is None:
            break
        ref.apply(psi, ref.matrix_of(g), g.qubits)
    return psi, outcomes
