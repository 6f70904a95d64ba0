"""Shared test helpers: input conversion only (no simulation arithmetic)."""
from __future__ import annotations

import os
import re

import numpy as np

from workloads.circuits import haar_unitary_from_seed

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def to_binding(gates):
    """workloads.Gate list -> tuples for the binding; MATRIX gates get their
    seeded input matrix."""
    out = []
    for g in gates:
        if g.name == "MATRIX":
            out.append(("MATRIX", g.qubits, (), g.param_index,
                        haar_unitary_from_seed(int(g.params[0]), len(g.qubits))))
        else:
            out.append((g.name, g.qubits, g.params, g.param_index))
    return out


def header_functions():
    """Names of the functions declared in include/*.h."""
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(sv_\w+)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return names


def fidelity_error(ref: np.ndarray, psi: np.ndarray) -> float:
    from oracle import ref as R
    return R.fidelity_error(ref, psi)
