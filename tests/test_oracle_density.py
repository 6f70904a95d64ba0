"""Pins of the density-matrix oracle (oracle/density.py) to closed forms,
to psi psi^dagger of the pinned state-vector oracle, and to the exact mixture
of sampled Pauli errors (paper, Noisy gates and Simulations with noise
sections; Gates and Properties section for the super-gate forms)."""
import itertools
import math

import numpy as np
import pytest

from oracle import density as dm
from oracle import ref
from workloads import circuits as wc
from workloads.circuits import Gate


def _rand_rho(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    rho = a @ a.conj().T
    return rho / np.trace(rho)


def test_pure_circuit_is_psi_psi_dagger():
    gates = wc.grid_rqc(2, 2, 6, seed=11)
    rho = dm.simulate(4, gates)
    psi = ref.simulate(4, gates, "0")
    assert np.abs(rho - dm.pure(psi)).max() < 1e-13


def test_depolarizing_closed_forms():
    p = 0.3
    rho = dm.apply_op(dm.zero(1), dm.depolarizing((0,), p))
    assert np.abs(rho - np.diag([1 - p / 2, p / 2])).max() < 1e-15
    r2 = _rand_rho(2, 5)
    out = dm.apply_op(r2, dm.depolarizing((0, 1), p))
    assert np.abs(out - ((1 - p) * r2 + p * np.eye(4) / 4)).max() < 1e-15
    # on one qubit of two: (1 - p) rho + p (I/2 (x) tr_q rho) with q = position 1
    out = dm.apply_op(r2, dm.depolarizing((1,), p))
    r = r2.reshape(2, 2, 2, 2)  # [q1, q0, q1', q0']
    tr1 = np.einsum("aiaj->ij", r)
    want = (1 - p) * r2 + p * np.kron(np.eye(2) / 2, tr1)
    assert np.abs(out - want).max() < 1e-15


def test_amplitude_damping_closed_form():
    # RX(-pi/2)|0> = (|0> + i|1>)/sqrt 2; damping gamma
    g = 0.37
    rho = dm.simulate(1, [Gate("RX", (0,), (-math.pi / 2,))], [dm.amplitude_damping(0, g, after=1)])
    want = np.array([[(1 + g) / 2, -1j * math.sqrt(1 - g) / 2],
                     [1j * math.sqrt(1 - g) / 2, (1 - g) / 2]])
    assert np.abs(rho - want).max() < 1e-15


@pytest.mark.parametrize("theta", [0.0, 0.7, 2.5])
def test_dephasing_of_rotating_spin(theta):
    # <X> = (1 - 2p) cos theta and <Y> = (1 - 2p) sin theta after H, RZ(theta), Z-dephasing p
    p = 0.2
    rho = dm.simulate(1, [Gate("H", (0,)), Gate("RZ", (0,), (theta,))], [dm.dephasing(0, p, after=2)])
    assert abs(dm.expectation(rho, [(1.0, ((0, "X"),))]) - (1 - 2 * p) * math.cos(theta)) < 1e-14
    assert abs(dm.expectation(rho, [(1.0, ((0, "Y"),))]) - (1 - 2 * p) * math.sin(theta)) < 1e-14
    assert abs(dm.expectation(rho, [(1.0, ())]) - 1.0) < 1e-14


def test_channel_equals_exact_mixture_of_sampled_paulis():
    # the trajectories' noise model: after each fSim, with probability p a
    # uniform two-qubit Pauli string (identity included)
    p = 0.05
    gates = wc.grid_rqc(1, 3, 4, seed=2)
    fs = [i for i, g in enumerate(gates) if g.name == "FSIM"][:3]
    gates = gates[:fs[-1] + 1]
    ops = [dm.depolarizing(gates[i].qubits, p, after=i + 1) for i in fs]
    rho = dm.simulate(3, gates, ops)
    want = np.zeros_like(rho)
    labels = ["".join(t) for t in itertools.product("IXYZ", repeat=2)]
    for pattern in itertools.product(range(16), repeat=len(fs)):
        w = 1.0
        seq = []
        for i, g in enumerate(gates):
            seq.append(g)
            if i in fs:
                code = pattern[fs.index(i)]
                w *= (1 - p) * (code == 0) + p / 16
                a, b = labels[code]
                if a != "I":
                    seq.append(Gate(a, (g.qubits[0],)))
                if b != "I":
                    seq.append(Gate(b, (g.qubits[1],)))
        want += w * dm.pure(ref.simulate(3, seq, "0"))
    assert np.abs(rho - want).max() < 1e-13


def test_matrix_super_gate_matches_kraus_form():
    # row-major vectorisation: vec(A rho B) = kron(A, B^T) vec(rho)
    rho = _rand_rho(3, 7)
    K = wc.random_kraus_from_seed(3, 2, 3)
    R = wc.random_kraus_from_seed(4, 2, 2)
    s = np.array([[0.3, 0.1j], [0.2, -0.4], [0.05, 0.5]])
    S = sum(s[i, j] * np.kron(K[i], R[j].conj()) for i in range(3) for j in range(2))
    for qs in [(0, 2), (2, 1)]:
        a = dm.apply_kraus_super(rho, K, R, s, qs)
        b = dm.apply_matrix_super(rho, S, qs)
        assert np.abs(a - b).max() < 1e-14


def test_random_channel_keeps_a_density_matrix():
    rho = _rand_rho(3, 9)
    for seed, (qs, m) in enumerate([((1,), 3), ((0, 2), 4), ((2, 0, 1), 2)]):
        out = dm.apply_op(rho, {"qubits": qs, "left": wc.random_kraus_from_seed(seed, len(qs), m)})
        assert abs(np.trace(out) - 1) < 1e-13
        assert np.abs(out - out.conj().T).max() < 1e-14
        assert np.linalg.eigvalsh(out).min() > -1e-13


def test_sampled_amplitude_damping_closed_form():
    g = 0.3
    K = dm.amplitude_damping(0, g)["left"]
    one = np.array([0, 1], dtype=np.complex128)
    p = dm.kraus_probabilities(one, K, (0,))
    assert abs(p[0] - (1 - g)) < 1e-15 and abs(p[1] - g) < 1e-15
    psi, i = dm.sample_kraus(one, K, (0,), 0.5)
    assert i == 0 and np.abs(psi - one).max() < 1e-15
    psi, i = dm.sample_kraus(one, K, (0,), 0.8)
    assert i == 1 and np.abs(psi - np.array([1, 0])).max() < 1e-15


def test_branches_of_sampled_channels_sum_to_the_density_matrix():
    # every outcome sequence, weighted by its probability, reproduces rho
    n = 3
    gates = wc.grid_rqc(1, 3, 3, seed=4)
    ops = [dm.amplitude_damping(0, 0.35, after=3),
           {"qubits": (2, 1), "left": wc.random_kraus_from_seed(8, 2, 3), "after": 6},
           dm.dephasing(1, 0.2, "X", after=len(gates))]
    rho = dm.simulate(n, gates, ops)

    def walk(psi, start, j, weight, acc):
        stop = ops[j]["after"] if j < len(ops) else len(gates)
        psi = psi.copy()
        for g in gates[start:stop]:
            ref.apply(psi, ref.matrix_of(g), g.qubits)
        if j == len(ops):
            acc += weight * dm.pure(psi)
            return
        p = dm.kraus_probabilities(psi, ops[j]["left"], ops[j]["qubits"])
        assert abs(sum(p) - 1) < 1e-13
        run = 0.0
        for i, w in enumerate(p):
            if w > 1e-15:
                u = (run + w / 2) / sum(p)  # the middle of outcome i's interval
                nxt, pick = dm.sample_kraus(psi, ops[j]["left"], ops[j]["qubits"], u)
                assert pick == i
                walk(nxt, stop, j + 1, weight * w, acc)
            run += w

    acc = np.zeros_like(rho)
    walk(ref.product_state(n, "0"), 0, 0, 1.0, acc)
    assert np.abs(acc - rho).max() < 1e-13


def test_trajectory_follows_the_drawn_branch():
    # dm.trajectory with given draws equals the branch built step by step from
    # kraus_probabilities and sample_kraus at the same places in the circuit
    n = 3
    gates = wc.grid_rqc(1, 3, 3, seed=4)
    ops = [dm.amplitude_damping(0, 0.35, after=3),
           {"qubits": (2, 1), "left": wc.random_kraus_from_seed(8, 2, 3), "after": 6},
           dm.dephasing(1, 0.2, "X", after=len(gates))]
    u = [0.9, 0.5, 0.1]
    psi, outcomes = dm.trajectory(n, gates, ops, u)
    want = ref.product_state(n, "0")
    start = 0
    for j, op in enumerate(ops):
        for g in gates[start:op["after"]]:
            ref.apply(want, ref.matrix_of(g), g.qubits)
        start = op["after"]
        want, pick = dm.sample_kraus(want, op["left"], op["qubits"], u[j])
        assert pick == outcomes[j]
    assert np.abs(psi - want).max() < 1e-14
    assert outcomes[0] == 1  # u = 0.9 jumps: the |1> weight after the first gates exceeds 0.1


def test_generalized_amplitude_damping_closed_forms():
    # populations: |0> -> diag(1 - b, b), |1> -> diag(g, 1 - g); coherences
    # shrink by sqrt((1 - b)(1 - g)); repeated application relaxes to the
    # population b / (b + g) of |1>
    g, b = 0.3, 0.12
    op = dm.amplitude_damping(0, g, b)
    assert np.abs(dm.apply_op(dm.zero(1), op) - np.diag([1 - b, b])).max() < 1e-15
    assert np.abs(dm.apply_op(np.diag([0, 1]).astype(complex), op) - np.diag([g, 1 - g])).max() < 1e-15
    plus = np.full((2, 2), 0.5, dtype=complex)
    out = dm.apply_op(plus, op)
    assert abs(out[0, 1] - 0.5 * math.sqrt((1 - b) * (1 - g))) < 1e-15
    assert abs(out[1, 0] - 0.5 * math.sqrt((1 - b) * (1 - g))) < 1e-15
    rho = plus
    for _ in range(300):
        rho = dm.apply_op(rho, op)
    assert abs(rho[1, 1].real - b / (b + g)) < 1e-13 and abs(rho[0, 1]) < 1e-13
    # excitation 0: the paper's two operators
    assert len(dm.amplitude_damping(0, g)["left"]) == 2


def test_pauli_channel_closed_forms():
    import scipy.linalg as sl
    # rank one, s = v v^dagger with v = cos a e_I - i sin a e_P: rho -> K rho K^dagger,
    # K = exp(-i a P) (P a Pauli string, P^2 = I)
    a = 0.37
    for qubits, label in (((0,), "Z"), ((1, 0), "XY"), ((0, 2, 1), "ZIX")):
        k = len(qubits)
        idx = sum("IXYZ".index(c) * 4 ** (k - 1 - j) for j, c in enumerate(label))
        v = np.zeros(4 ** k, dtype=complex)
        v[0], v[idx] = math.cos(a), -1j * math.sin(a)
        rho = _rand_rho(3, 21)
        out = dm.apply_op(rho, dm.pauli_channel(qubits, np.outer(v, v.conj())))
        P = dm.pauli_string(label)
        K = sl.expm(-1j * a * P)
        want = dm.apply_kraus_super(rho, [K], [K], None, qubits)
        assert np.abs(out - want).max() < 1e-14
    # rank one on a single qubit against the rotation of the gate table:
    # exp(-i a Z) = RZ(2a)
    rho = _rand_rho(1, 22)
    v = np.array([math.cos(a), 0, 0, -1j * math.sin(a)])
    out = dm.apply_op(rho, dm.pauli_channel((0,), np.outer(v, v.conj())))
    assert np.abs(out - dm.apply_gate(rho, ref.gate_matrix("RZ", (2 * a,)), (0,))).max() < 1e-15
    # diagonal s: Z dephasing, off-diagonals times (1 - 2p)
    p = 0.15
    out = dm.apply_op(rho, dm.pauli_channel((0,), np.diag([1 - p, 0, 0, p])))
    assert np.abs(out - np.array([[rho[0, 0], (1 - 2 * p) * rho[0, 1]],
                                  [(1 - 2 * p) * rho[1, 0], rho[1, 1]]])).max() < 1e-15
    # the depolarizing weights as a diagonal s give the depolarizing channel
    d2 = 16
    w = np.full(d2, 0.2 / d2)
    w[0] += 0.8
    r2 = _rand_rho(2, 23)
    assert np.abs(dm.apply_op(r2, dm.pauli_channel((0, 1), np.diag(w)))
                  - ((1 - 0.2) * r2 + 0.2 * np.eye(4) / 4)).max() < 1e-15
