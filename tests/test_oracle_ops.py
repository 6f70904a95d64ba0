"""Pins of oracle/ops.py: the paper's Grover example (printed values), textbook
controlled gates, and projections / measurements of states with known
outcomes (GHZ) and the Born rule by brute force."""
import os

import numpy as np
import pytest

from oracle import ops, ref

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden_grover():
    rows = []
    for line in open(os.path.join(HERE, "golden", "grover_3q.txt")):
        if line.strip() and not line.startswith("#"):
            b, v = line.split()
            rows.append((b, float(v)))
    return rows


def test_grover_oracle_by_projection_matches_the_paper():
    # order = [0, 1, 2]: paper qubit j is position 2 - j; the gate acts on paper qubits 1, 2
    psi = ref.product_state(3, "+")
    psi0, p = ops.project(psi, (1, 0), "00", renormalize=False)
    out = psi - 2 * psi0
    assert abs(p - 0.25) < 1e-15
    for b, v in _golden_grover():
        assert abs(out[int(b, 2)].real - v) < 5e-7 and abs(out[int(b, 2)].imag) < 1e-15


def test_controlled_gates_are_the_textbook_ones():
    X, Z = ref.gate_matrix("X"), ref.gate_matrix("Z")
    assert np.abs(ops.controlled(X, 1) - ref.gate_matrix("CX")).max() == 0
    assert np.abs(ops.controlled(Z, 1) - ref.gate_matrix("CZ")).max() == 0
    T = ops.controlled(X, 2)  # Toffoli: flips the target only on 11x
    for x in range(8):
        y = x ^ 1 if x >> 1 == 3 else x
        assert T[y, x] == 1


def test_measure_ghz_collapses():
    ghz = np.zeros(8, dtype=np.complex128)
    ghz[0] = ghz[7] = 1 / np.sqrt(2)
    psi, bits, p = ops.measure(ghz, (0,), [0.3])
    assert bits == "0" and abs(p - 0.5) < 1e-15 and abs(abs(psi[0]) - 1) < 1e-15
    psi, bits, p = ops.measure(ghz, (2,), [0.7])
    assert bits == "1" and abs(p - 0.5) < 1e-15 and abs(abs(psi[7]) - 1) < 1e-15
    psi, bits, p = ops.measure(ghz, (2, 0, 1), [0.7, 0.1, 0.9])
    assert bits == "111" and abs(p - 0.5) < 1e-15


def test_born_rule_by_brute_force():
    rng = np.random.default_rng(4)
    psi = rng.standard_normal(32) + 1j * rng.standard_normal(32)
    psi /= np.linalg.norm(psi)
    qs = (3, 0, 4)
    for bits in ("000", "101", "110"):
        _, p = ops.project(psi, qs, bits, renormalize=False)
        want = sum(abs(psi[i]) ** 2 for i in range(32)
                   if all(((i >> q) & 1) == int(b) for q, b in zip(qs, bits)))
        assert abs(p - want) < 1e-15
    # sequential measurement reproduces the joint probability
    _, bits, p = ops.measure(psi, qs, [0.2, 0.6, 0.9])
    _, pj = ops.project(psi, qs, bits, renormalize=False)
    assert abs(p - pj) < 1e-14
