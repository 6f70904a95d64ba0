"""Seeded circuit generators for the synthetic workloads.

A circuit is an ordered list of gates acting on qubits (Circuits section of
the paper).  Qubits here are *positions*: position p is bit p of an amplitude
index (position 0 is the least significant bit).  Grid site (r, c) of an
R x C grid is position r*C + c.

Random-circuit structure.  The paper times random circuits from a generator it
does not define (State Vector section, the timing table for 12..28 qubits); the
synthetic circuits below stand in for them:

* cycle l = one single-qubit layer on every qubit, then fSim(pi/2, pi/6) on the
  nearest-neighbour edge set S[l mod 4]; no trailing single-qubit layer;
* S0 / S1 = horizontal edges (r,c)-(r,c+1) with r+c even / odd,
  S2 / S3 = vertical edges (r,c)-(r+1,c) with r+c even / odd;
* the single-qubit gate is uniform over {sqrt(X), sqrt(Y), sqrt(W)} in cycle 0,
  afterwards uniform over the two gates different from the previous one on
  that qubit; draws are made qubit by qubit in position order, cycle by cycle,
  from ``numpy.random.default_rng(seed)``.

Noisy trajectories (Simulations with noise section; the global depolarizing
channel of the Noisy gates section applied to the two qubits of each two-qubit
gate): after every fSim, with probability p a uniform draw from the 16
two-qubit Pauli strings (identity included) is inserted.  The channel
rho -> (1-p) rho + p I/4 on two qubits is exactly this mixture.  Identity
factors are not emitted as gates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ONE_QUBIT_SET = ("SQRT_X", "SQRT_Y", "SQRT_W")
FSIM_THETA = math.pi / 2
FSIM_PHI = math.pi / 6


@dataclass(frozen=True)
class Gate:
    """One gate: a name from the shared vocabulary, the qubit positions it acts
    on (``qubits[0]`` is the most significant bit of the gate's local index),
    its real parameters and, for differentiable rotations, the index of its
    parameter in the parameter vector (-1 otherwise)."""

    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    param_index: int = -1


def grid_edge_sets(rows: int, cols: int) -> List[List[Tuple[int, int]]]:
    """The four nearest-neighbour matchings S0..S3 of an R x C grid."""
    sets: List[List[Tuple[int, int]]] = [[], [], [], []]
    for r in range(rows):
        for c in range(cols - 1):
            sets[0 if (r + c) % 2 == 0 else 1].append((r * cols + c, r * cols + c + 1))
    for r in range(rows - 1):
        for c in range(cols):
            sets[2 if (r + c) % 2 == 0 else 3].append((r * cols + c, (r + 1) * cols + c))
    return sets


def _rqc_on_sites(sites: Sequence[int], edge_sets, depth: int, rng) -> List[Gate]:
    gates: List[Gate] = []
    prev = {q: -1 for q in sites}
    for cycle in range(depth):
        for q in sites:
            if prev[q] < 0:
                choice = int(rng.integers(3))
            else:
                others = [i for i in range(3) if i != prev[q]]
                choice = others[int(rng.integers(2))]
            prev[q] = choice
            gates.append(Gate(ONE_QUBIT_SET[choice], (q,)))
        for (a, b) in edge_sets[cycle % 4]:
            gates.append(Gate("FSIM", (a, b), (FSIM_THETA, FSIM_PHI)))
    return gates


def grid_rqc(rows: int, cols: int, depth: int, seed: int) -> List[Gate]:
    """Random circuit on an R x C grid (see module docstring)."""
    rng = np.random.default_rng(seed)
    return _rqc_on_sites(list(range(rows * cols)), grid_edge_sets(rows, cols), depth, rng)


def ladder_rqc(n: int, depth: int, rng) -> List[Gate]:
    """Random circuit on a 2 x ceil(n/2) ladder; for odd n the site (1, C-1) is
    absent and every edge touching it is dropped.  Positions are renumbered
    densely in site order so the circuit acts on positions 0..n-1."""
    cols = (n + 1) // 2
    present = [r * cols + c for r in range(2) for c in range(cols)]
    if n % 2 == 1:
        present.remove(1 * cols + cols - 1)
    dense = {s: i for i, s in enumerate(present)}
    sets = []
    for es in grid_edge_sets(2, cols):
        sets.append([(dense[a], dense[b]) for (a, b) in es if a in dense and b in dense])
    return _rqc_on_sites(list(range(n)), sets, depth, rng)


# The three grid workloads: (rows, cols, depth, seed).
GRID_CONFIGS = {
    0: (2, 7, 12, 0),   # 14 qubits, 225 gates
    1: (5, 6, 20, 1),   # 30 qubits, 845 gates
    2: (4, 8, 14, 2),   # 32 qubits, 632 gates
}


def config_circuit(i: int) -> Tuple[int, List[Gate]]:
    rows, cols, depth, seed = GRID_CONFIGS[i]
    return rows * cols, grid_rqc(rows, cols, depth, seed)


def ansatz_circuit(n: int = 20, layers: int = 12, seed: int = 3):
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every
    qubit, then CZ(i, i+1) for i = 0..n-2.  The parameter of RY on qubit q in
    layer l has index l*2n + q, RZ has l*2n + n + q.  Angles are uniform on
    [0, 2 pi) from ``default_rng(seed)``.  Returns (gates, thetas)."""
    rng = np.random.default_rng(seed)
    thetas = rng.uniform(0.0, 2.0 * math.pi, size=layers * 2 * n)
    gates: List[Gate] = []
    for layer in range(layers):
        for q in range(n):
            p = layer * 2 * n + q
            gates.append(Gate("RY", (q,), (float(thetas[p]),), p))
        for q in range(n):
            p = layer * 2 * n + n + q
            gates.append(Gate("RZ", (q,), (float(thetas[p]),), p))
        for q in range(n - 1):
            gates.append(Gate("CZ", (q, q + 1)))
    return gates, thetas


def ansatz_observable(n: int = 20):
    """H = sum_i Z_i Z_{i+1} + 0.5 sum_i X_i on an open chain, as a list of
    (coefficient, ((position, pauli), ...))."""
    terms = [(1.0, ((i, "Z"), (i + 1, "Z"))) for i in range(n - 1)]
    terms += [(0.5, ((i, "X"),)) for i in range(n)]
    return terms


def with_thetas(gates: Sequence[Gate], thetas) -> List[Gate]:
    """Rebind the angles of differentiable rotations to ``thetas``."""
    out = []
    for g in gates:
        if g.param_index >= 0:
            out.append(Gate(g.name, g.qubits, (float(thetas[g.param_index]),), g.param_index))
        else:
            out.append(g)
    return out


PAULI_LABELS = ("I", "X", "Y", "Z")


@dataclass
class Trajectory:
    n: int
    depth: int
    gates: List[Gate] = field(default_factory=list)
    n_inserted: int = 0


def trajectory_batch(count: int = 512, root_seed: int = 4, p: float = 1e-3,
                     n_range=(10, 22), depth_range=(8, 24),
                     noise: bool = True) -> List[Trajectory]:
    """Noisy-trajectory batch.  Trajectory t draws from
    ``default_rng(SeedSequence(root_seed).spawn(count)[t])``: first n, then the
    depth, then all of the circuit's single-qubit choices cycle by cycle, then,
    for each fSim in circuit order, one uniform in [0,1) and, when it falls
    below p, one integer in 0..15 choosing the two-qubit Pauli (the 4s digit
    is the factor on the gate's first qubit)."""
    children = np.random.SeedSequence(root_seed).spawn(count)
    batch = []
    for t in range(count):
        rng = np.random.default_rng(children[t])
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        clean = _ladder_with_rng(n, depth, rng)
        gates: List[Gate] = []
        inserted = 0
        for g in clean:
            gates.append(g)
            if g.name == "FSIM" and noise:
                u = float(rng.random())
                if u < p:
                    code = int(rng.integers(16))
                    a, b = PAULI_LABELS[code // 4], PAULI_LABELS[code % 4]
                    if a != "I":
                        gates.append(Gate(a, (g.qubits[0],)))
                    if b != "I":
                        gates.append(Gate(b, (g.qubits[1],)))
                    inserted += 1
        batch.append(Trajectory(n, depth, gates, inserted))
    return batch


def _ladder_with_rng(n: int, depth: int, rng) -> List[Gate]:
    return ladder_rqc(n, depth, rng)


def paper_compress_example() -> List[Gate]:
    """The circuit of the paper's compress example (Circuit utilities
    section): CPHASE(1) on every pair q1 < q2 of 5 qubits, q1 outer loop."""
    return [Gate("CPHASE", (q1, q2), (1.0,)) for q1 in range(5) for q2 in range(q1 + 1, 5)]


def qubit_names_to_positions(order: Sequence, qubits: Sequence) -> Tuple[int, ...]:
    """Map named qubits to positions under the paper's array convention: axis
    j of a ``(2,)*n`` state follows ``order[j]`` and the ravel is C-order, so
    ``order[0]`` is the most significant bit, position n-1."""
    n = len(order)
    index = {name: j for j, name in enumerate(order)}
    return tuple(n - 1 - index[q] for q in qubits)


def random_gate_list(n: int, count: int, rng, max_k: int = 3,
                     names: Optional[Sequence[str]] = None) -> List[Gate]:
    """Random mixed-arity gate list for parity tests: named gates and dense
    random unitaries ('MATRIX' gates carry a seed for the matrix draw in
    params[0]; the matrix itself is built by whichever side consumes it)."""
    names = names or ("H", "SQRT_X", "SQRT_Y", "SQRT_W", "RX", "RY", "RZ",
                      "CZ", "CX", "CPHASE", "FSIM", "SWAP", "MATRIX")
    one_q = {"H", "SQRT_X", "SQRT_Y", "SQRT_W", "RX", "RY", "RZ", "X", "Y", "Z"}
    two_q = {"CZ", "CX", "CPHASE", "FSIM", "SWAP"}
    gates = []
    for _ in range(count):
        name = names[int(rng.integers(len(names)))]
        if name in one_q:
            k = 1
        elif name in two_q:
            k = 2
        else:
            k = int(rng.integers(1, min(max_k, n) + 1))
        if k > n:
            continue
        qs = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        if name in ("RX", "RY", "RZ", "CPHASE"):
            params = (float(rng.uniform(0, 2 * math.pi)),)
        elif name == "FSIM":
            params = (float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(0, 2 * math.pi)))
        elif name == "MATRIX":
            params = (float(rng.integers(1 << 30)),)
        else:
            params = ()
        gates.append(Gate(name, qs, params))
    return gates


def haar_unitary_from_seed(seed: int, k: int) -> np.ndarray:
    """Input generator for 'MATRIX' gates: a Haar-random 2^k x 2^k unitary from
    the QR of a complex Gaussian matrix (Mezzadri's recipe).  This is an input
    drawn once; both sides receive the same matrix."""
    rng = np.random.default_rng(int(seed))
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def random_kraus_from_seed(seed: int, k: int, n_ops: int) -> List[np.ndarray]:
    """Input generator for Kraus channels: n_ops operators K_i (2^k x 2^k) with
    sum_i K_i^dagger K_i = I, the blocks of a random isometry (QR of a complex
    Gaussian (n_ops 2^k) x 2^k matrix).  Both sides receive the same operators."""
    rng = np.random.default_rng(int(seed))
    d = 1 << k
    z = (rng.standard_normal((n_ops * d, d)) + 1j * rng.standard_normal((n_ops * d, d))) / math.sqrt(2)
    v, _ = np.linalg.qr(z)
    return [np.ascontiguousarray(v[i * d:(i + 1) * d, :]) for i in range(n_ops)]


def noisy_grid_circuit(rows: int, cols: int, depth: int, seed: int, p: float = 1e-3):
    """Density-matrix workload: the grid random circuit with the two-qubit
    global depolarizing channel (probability p) after every fSim.  Returns
    (gates, channels) where a channel is (after, qubits, p): it acts after the
    first ``after`` gates."""
    gates = grid_rqc(rows, cols, depth, seed)
    channels = [(i + 1, g.qubits, p) for i, g in enumerate(gates) if g.name == "FSIM"]
    return gates, channels


def pauli_trajectories(gates: Sequence[Gate], p: float, count: int, seed: int) -> List[List[Gate]]:
    """``count`` samples of the fixed circuit ``gates`` under the trajectories'
    noise model: after every fSim, with probability p, a uniform draw from the
    16 two-qubit Pauli strings (identity included) is inserted."""
    rng = np.random.default_rng(int(seed))
    out = []
    for _ in range(count):
        seq: List[Gate] = []
        for g in gates:
            seq.append(g)
            if g.name == "FSIM" and float(rng.random()) < p:
                code = int(rng.integers(16))
                a, b = PAULI_LABELS[code // 4], PAULI_LABELS[code % 4]
                if a != "I":
                    seq.append(Gate(a, (g.qubits[0],)))
                if b != "I":
                    seq.append(Gate(b, (g.qubits[1],)))
        out.append(seq)
    return out
