"""Oracle: projection, measurement and controlled gates -- TEST INFRASTRUCTURE ONLY.

Only tests use this module; it shares no code with the HIP library.  Plain
definitions (paper, Gates and Properties section: Projection(state, qubits),
Measure(qubits), Control(c_qubits, gate); Grover Oracle section: the oracle
is psi - 2 P psi with P the projection on |0..0>), in complex128 through the
state-vector oracle's ``apply``.  Pins: tests/test_oracle_ops.py.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import ref


def projector(bits: str) -> np.ndarray:
    """|bits><bits| (bits[0] the most significant local bit)."""
    d = 1 << len(bits)
    P = np.zeros((d, d), dtype=np.complex128)
    i = int(bits, 2)
    P[i, i] = 1.0
    return P


def project(psi: np.ndarray, qubits: Sequence[int], bits: str, renormalize: bool = True):
    out = ref.apply(psi.copy(), projector(bits), qubits)
    p = ref.norm2(out)
    if renormalize:
        out = out / np.sqrt(p)
    return out, p


def measure(psi: np.ndarray, qubits: Sequence[int], uniforms):
    """Qubit by qubit: outcome 0 when u < p0 / (p0 + p1), else 1 (an outcome of
    zero weight is never taken); the state collapses and is renormalised."""
    bits, ptot = "", 1.0
    for q, u in zip(qubits, uniforms):
        p0 = ref.norm2(ref.apply(psi.copy(), projector("0"), (q,)))
        p1 = ref.norm2(ref.apply(psi.copy(), projector("1"), (q,)))
        b = 0 if (p0 > 0 and u * (p0 + p1) < p0) or p1 == 0 else 1
        pb = p1 if b else p0
        psi = ref.apply(psi.copy(), projector(str(b)), (q,)) / np.sqrt(pb)
        bits += str(b)
        ptot *= pb / (p0 + p1)
    return psi, bits, ptot


def controlled(U: np.ndarray, n_c: int) -> np.ndarray:
    """I (+) ... (+) U: U acts when all n_c controls (the most significant
    local bits) are 1."""
    d = U.shape[0]
    D = d << n_c
    C = np.eye(D, dtype=np.complex128)
    C[D - d:, D - d:] = U
    return C
