"""Brute force: the full 2^n x 2^n unitary of a circuit, n <= 8 -- TEST
INFRASTRUCTURE ONLY.

This is the paper's ``matrix(circuit)`` utility (Circuit utilities section)
written with Kronecker products, independently of the index arithmetic in
``ref.apply``: a k-qubit gate M on qubits q is

    sum_{a,b} M[a,b]  (x)_{p = n-1 .. 0}  F_p,
    F_p = |a_j><b_j|  if p = q_j  (a_j = bit k-1-j of a),  else  I,

where the Kronecker product runs from position n-1 (most significant) down to
position 0, and the circuit unitary is the ordered product U_G ... U_1.
"""
from __future__ import annotations

from functools import reduce
from typing import Sequence, Tuple

import numpy as np

MAX_N = 8


def _unit(a: int, b: int) -> np.ndarray:
    E = np.zeros((2, 2), dtype=np.complex128)
    E[a, b] = 1.0
    return E


def embed(n: int, M: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    assert n <= MAX_N
    k = len(qubits)
    D = 1 << k
    I2 = np.eye(2, dtype=np.complex128)
    U = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    where = {q: j for j, q in enumerate(qubits)}
    for a in range(D):
        for b in range(D):
            if M[a, b] == 0:
                continue
            factors = []
            for p in range(n - 1, -1, -1):
                if p in where:
                    j = where[p]
                    factors.append(_unit((a >> (k - 1 - j)) & 1, (b >> (k - 1 - j)) & 1))
                else:
                    factors.append(I2)
            U += M[a, b] * reduce(np.kron, factors)
    return U


def circuit_unitary(n: int, ops: Sequence[Tuple[np.ndarray, Sequence[int]]]) -> np.ndarray:
    U = np.eye(1 << n, dtype=np.complex128)
    for M, q in ops:
        U = embed(n, np.asarray(M, dtype=np.complex128), q) @ U
    return U


def pauli_string_matrix(n: int, factors) -> np.ndarray:
    """Kronecker product of single-qubit Paulis (identity elsewhere)."""
    P = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]),
         "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.array([[1, 0], [0, -1]])}
    at = {q: p for q, p in factors}
    return reduce(np.kron, [np.asarray(P[at.get(p, "I")], dtype=np.complex128)
                            for p in range(n - 1, -1, -1)])


def observable_matrix(n: int, terms) -> np.ndarray:
    return sum(c * pauli_string_matrix(n, f) for c, f in terms)
