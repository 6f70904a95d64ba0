"""Pins that tie the oracle to the paper and to mathematics.

Each ``check_*`` raises AssertionError when the oracle disagrees with the fixed
fact it encodes.  They are called by test_oracle_pins.py and, with mistakes
planted into the oracle, by test_oracle_mutants.py (each planted mistake must
trip at least one pin).
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.linalg

from oracle import brute, ref
from workloads import circuits as wc
from workloads.circuits import Gate

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


# ---------------------------------------------------------------- paper examples
def check_grover_worked_example():
    """Grover Oracle section: the FunctionalGate computes psi - 2 P00 psi on
    qubits [1, 2] of the uniform 3-qubit state, order = [0, 1, 2]; as a matrix
    on those qubits that is I - 2|00><00|."""
    order = [0, 1, 2]
    psi = ref.product_state(3, "+")
    proj00 = np.zeros((4, 4), dtype=complex)
    proj00[0, 0] = 1.0
    D = np.eye(4) - 2 * proj00
    ref.apply(psi, D, wc.qubit_names_to_positions(order, [1, 2]))
    got = {format(i, "03b"): psi[i] for i in range(8)}
    for bits, val in _golden_lines("grover_3q.txt"):
        assert abs(got[bits].imag) < 1e-15
        assert abs(got[bits].real - float(val)) < 5e-7, (bits, got[bits], val)


def check_compress_worked_example():
    """Circuit utilities section: compress(max_n_qubits=3) of CPHASE on all
    pairs of 5 qubits yields blocks (0,1,2), (0,3,4), (1,3,4), (2,3,4)."""
    gates = wc.paper_compress_example()
    blocks = ref.fuse_paper([g.qubits for g in gates], 3)
    want = [tuple(int(x) for x in ln) for ln in _golden_lines("compress_cphase5_k3.txt")]
    assert [b[0] for b in blocks] == want, blocks


# ---------------------------------------------------------------- brute force
def _random_ops(n, count, rng, max_k=3):
    gates = wc.random_gate_list(n, count, rng, max_k=max_k)
    return gates, [(ref.matrix_of(g), g.qubits) for g in gates]


def _random_tokens(n, rng):
    return "".join("01+-"[int(x)] for x in rng.integers(4, size=n))


def check_apply_vs_brute(seed=0, max_n=8, max_k=3):
    rng = np.random.default_rng(seed)
    for n in range(1, max_n + 1):
        for _ in range(3):
            gates, ops = _random_ops(n, 12, rng, max_k=min(max_k, n))
            tokens = _random_tokens(n, rng)
            psi0 = ref.product_state(n, tokens)
            want = brute.circuit_unitary(n, ops) @ psi0
            got = ref.simulate(n, gates, tokens)
            assert np.max(np.abs(got - want)) <= 1e-13, (n, np.max(np.abs(got - want)))


def check_large_k_vs_brute(seed=1):
    """Dense k = 4..6 blocks at arbitrary positions (the shapes fusion makes)."""
    rng = np.random.default_rng(seed)
    for n, k in ((6, 4), (7, 5), (8, 6), (8, 4)):
        qs = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        M = wc.haar_unitary_from_seed(int(rng.integers(1 << 30)), k)
        psi0 = ref.product_state(n, _random_tokens(n, rng))
        want = brute.embed(n, M, qs) @ psi0
        got = ref.apply(psi0.copy(), M, qs)
        assert np.max(np.abs(got - want)) <= 1e-13


# ---------------------------------------------------------------- closed forms
def check_ghz(max_n=12):
    """H(0), CX(0,1), ..., CX(n-2, n-1) prepares (|0..0> + |1..1>)/sqrt 2; the
    control of CX is its first qubit."""
    for n in range(2, max_n + 1):
        gates = [Gate("H", (0,))] + [Gate("CX", (i, i + 1)) for i in range(n - 1)]
        psi = ref.simulate(n, gates, "0")
        want = np.zeros(1 << n, dtype=complex)
        want[0] = want[-1] = 1 / math.sqrt(2)
        assert np.max(np.abs(psi - want)) <= 1e-15 * 8


def qft_gates(n):
    """Textbook QFT with bit reversal at the end: for j = n-1..0: H(j), then
    controlled phases 2 pi / 2^(j-m+1) between j and each m < j; then swaps."""
    gates = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("H", (j,)))
        for m in range(j - 1, -1, -1):
            gates.append(Gate("CPHASE", (j, m), (2 * math.pi / 2 ** (j - m + 1),)))
    for j in range(n // 2):
        gates.append(Gate("SWAP", (j, n - 1 - j)))
    return gates


def check_qft_basis_states(max_n=8, seed=2):
    """QFT|x> = N^{-1/2} sum_y exp(2 pi i x y / N) |y>: exact phases."""
    rng = np.random.default_rng(seed)
    for n in range(1, max_n + 1):
        N = 1 << n
        for x in {0, N - 1, int(rng.integers(N)), int(rng.integers(N))}:
            psi = ref.simulate(n, qft_gates(n), psi=ref.basis_state(n, x))
            y = np.arange(N)
            want = np.exp(2j * math.pi * x * y / N) / math.sqrt(N)
            assert np.max(np.abs(psi - want)) <= 1e-13, (n, x)


def check_gate_table():
    names1 = ["I", "X", "Y", "Z", "H", "SQRT_X", "SQRT_Y", "SQRT_W"]
    for nm in names1 + ["CZ", "CX", "SWAP"]:
        M = ref.gate_matrix(nm)
        assert np.allclose(M.conj().T @ M, np.eye(M.shape[0]), atol=1e-15)
    for nm, P in (("RX", "X"), ("RY", "Y"), ("RZ", "Z")):
        for th in (0.3, 2.1, -4.0):
            M = ref.gate_matrix(nm, (th,))
            assert np.allclose(M.conj().T @ M, np.eye(2), atol=1e-15)
    # (sqrt P)^2 = P, and the principal branch: scipy's principal square root
    X, Y = ref.PAULI["X"], ref.PAULI["Y"]
    W = (X + Y) / math.sqrt(2)
    for nm, P in (("SQRT_X", X), ("SQRT_Y", Y), ("SQRT_W", W)):
        S = ref.gate_matrix(nm)
        assert np.allclose(S @ S, P, atol=1e-15)
        assert np.allclose(S, scipy.linalg.sqrtm(P), atol=1e-12)
    # fSim(pi/2, 0)|01> = -i|10>; fSim(0, phi) = diag(1,1,1,e^{-i phi})
    F = ref.gate_matrix("FSIM", (math.pi / 2, 0.0))
    v = np.zeros(4, dtype=complex); v[1] = 1
    want = np.zeros(4, dtype=complex); want[2] = -1j
    assert np.allclose(F @ v, want, atol=1e-15)
    assert np.allclose(ref.gate_matrix("FSIM", (0.0, 0.7)), np.diag([1, 1, 1, np.exp(-0.7j)]))
    # CPHASE(pi) = CZ
    assert np.allclose(ref.gate_matrix("CPHASE", (math.pi,)), ref.gate_matrix("CZ"), atol=1e-15)
    # Gates and Properties section: RX(pi)**2.2 is the rotation by 2.2 pi
    # (matrix power on the principal branch).  This fixes the factor 1/2 in
    # R(theta) = exp(-i theta P / 2).
    for nm in ("RX", "RY", "RZ"):
        Mp = scipy.linalg.fractional_matrix_power(ref.gate_matrix(nm, (math.pi,)), 2.2)
        assert np.allclose(Mp, ref.gate_matrix(nm, (2.2 * math.pi,)), atol=1e-12)
    # RY(theta)|0>: <Z> = cos(theta), <X> = sin(theta)
    for th in (0.0, 0.4, 1.9, 3.7, -2.2):
        psi = ref.simulate(1, [Gate("RY", (0,), (th,))], "0")
        assert abs(ref.expectation(psi, [(1.0, ((0, "Z"),))]) - math.cos(th)) < 1e-15
        assert abs(ref.expectation(psi, [(1.0, ((0, "X"),))]) - math.sin(th)) < 1e-15
    # RZ(theta) = diag(e^{-i theta/2}, e^{i theta/2})
    assert np.allclose(ref.gate_matrix("RZ", (0.9,)), np.diag([np.exp(-0.45j), np.exp(0.45j)]))


def check_product_states(seed=3):
    r = 1 / math.sqrt(2)
    vec = {"0": [1, 0], "1": [0, 1], "+": [r, r], "-": [r, -r]}
    for n in range(1, 11):
        psi = ref.product_state(n, "+")
        assert np.max(np.abs(psi - 2.0 ** (-n / 2))) <= 1e-15
    rng = np.random.default_rng(seed)
    for n in range(1, 9):
        tok = _random_tokens(n, rng)
        want = np.array([1.0 + 0j])
        for t in tok:  # token 0 is the most significant qubit
            want = np.kron(want, np.array(vec[t], dtype=complex))
        assert np.max(np.abs(ref.product_state(n, tok) - want)) <= 1e-15


# ---------------------------------------------------------------- invariants
def check_norm_and_reversibility(seed=4):
    rng = np.random.default_rng(seed)
    for n in (6, 10, 12):
        gates = wc.random_gate_list(n, 80, rng, max_k=3)
        psi0 = ref.product_state(n, _random_tokens(n, rng))
        psi = ref.simulate(n, gates, psi=psi0.copy())
        assert abs(ref.norm2(psi) - 1.0) <= 1e-12
        back = ref.run_matrices(psi.copy(), ref.inverse_ops(gates))
        assert np.max(np.abs(back - psi0)) <= 1e-12
    n, gates = wc.config_circuit(0)
    psi = ref.simulate(n, gates, "0")
    assert abs(ref.norm2(psi) - 1.0) <= 1e-12
    back = ref.run_matrices(psi.copy(), ref.inverse_ops(gates))
    assert np.max(np.abs(back - ref.basis_state(n, 0))) <= 1e-12


def check_fusion_product(seed=5):
    """A fused plan (paper rule) applied block by block reproduces the circuit's
    brute-force unitary, for every block size limit."""
    rng = np.random.default_rng(seed)
    for n in (4, 6, 7):
        gates = wc.random_gate_list(n, 30, rng, max_k=2)
        ops = [(ref.matrix_of(g), g.qubits) for g in gates]
        U = brute.circuit_unitary(n, ops)
        for k in range(2, min(n, 6) + 1):
            plan = ref.fuse_paper([g.qubits for g in gates], k)
            assert sorted(i for _, m in plan for i in m) == list(range(len(gates)))
            fused = []
            for qs, members in plan:
                assert len(qs) <= k
                assert all(set(gates[i].qubits) <= set(qs) for i in members)
                assert members == sorted(members)
                fused.append((ref.block_matrix([ops[i] for i in members], qs), qs))
            assert np.max(np.abs(brute.circuit_unitary(n, fused) - U)) <= 1e-12


def check_expectation(seed=6):
    rng = np.random.default_rng(seed)
    # basis states: Z strings give (-1)^{popcount(x & S)}
    for n in (3, 5):
        for _ in range(6):
            x = int(rng.integers(1 << n))
            S = [q for q in range(n) if rng.random() < 0.5]
            want = (-1) ** bin(x & sum(1 << q for q in S)).count("1")
            e = ref.expectation(ref.basis_state(n, x), [(1.0, tuple((q, "Z") for q in S))])
            assert abs(e - want) < 1e-15
    # product states: <X> = +-1 on |+->, <Z> = 0 there, <Y> = 0 on all tokens
    psi = ref.product_state(3, "+-0")   # positions 2:'+', 1:'-', 0:'0'
    assert abs(ref.expectation(psi, [(1.0, ((2, "X"),))]) - 1) < 1e-15
    assert abs(ref.expectation(psi, [(1.0, ((1, "X"),))]) + 1) < 1e-15
    assert abs(ref.expectation(psi, [(1.0, ((0, "Z"),))]) - 1) < 1e-15
    assert abs(ref.expectation(psi, [(2.5, ((2, "X"), (0, "Z")))]) - 2.5) < 1e-15
    assert abs(ref.expectation(psi, [(1.0, ((2, "Z"),))])) < 1e-15
    # brute force psi^dagger H psi for random states and sums with Y factors
    for n in (2, 4, 6):
        gates = wc.random_gate_list(n, 20, rng, max_k=2)
        psi = ref.simulate(n, gates, "0")
        terms = []
        for _ in range(5):
            f = tuple((q, "XYZ"[int(rng.integers(3))]) for q in range(n) if rng.random() < 0.6)
            terms.append((float(rng.normal()), f))
        want = np.vdot(psi, brute.observable_matrix(n, terms) @ psi).real
        assert abs(ref.expectation(psi, terms) - want) < 1e-13


def _small_ansatz(n=4, layers=2, seed=7):
    gates, thetas = wc.ansatz_circuit(n, layers, seed)
    return gates, thetas, wc.ansatz_observable(n)


def check_gradients():
    # one rotation: E = <Z> after RY(theta)|0> = cos(theta)
    for th in (0.3, 1.7, 4.0):
        g = ref.param_shift_grad(1, [Gate("RY", (0,), (th,), 0)], [th], [(1.0, ((0, "Z"),))])
        assert abs(g[0] + math.sin(th)) < 1e-14
    # ansatz: E(theta_p) = A + B cos + C sin exactly; recover the derivative from
    # three brute-force energies and compare with parameter shift; FD = g sinc(h)
    gates, thetas, H = _small_ansatz()
    n = 4
    Hm = brute.observable_matrix(n, H)

    def e_brute(th):
        ops = [(ref.matrix_of(g), g.qubits) for g in wc.with_thetas(gates, th)]
        psi = brute.circuit_unitary(n, ops)[:, 0]
        return np.vdot(psi, Hm @ psi).real

    ps = ref.param_shift_grad(n, gates, thetas, H)
    h = 1e-3
    fd = ref.fd_grad(n, gates, thetas, H, h=h)
    for p in range(len(thetas)):
        t0 = thetas[p]
        angles = [t0, t0 + 2 * math.pi / 3, t0 + 4 * math.pi / 3]
        es = []
        for a in angles:
            th = thetas.copy(); th[p] = a
            es.append(e_brute(th))
        A = np.array([[1, math.cos(a), math.sin(a)] for a in angles])
        _, B, C = np.linalg.solve(A, np.array(es))
        exact = -B * math.sin(t0) + C * math.cos(t0)
        assert abs(ps[p] - exact) < 1e-12, (p, ps[p], exact)
        assert abs(fd[p] - exact * math.sin(h) / h) < 1e-9, (p, fd[p], exact)


def check_trajectories():
    """Noisy gates (Noisy gates section): the two-qubit depolarizing channel
    rho -> (1-p) rho + p I/4 is the uniform mixture over the 16 two-qubit Pauli
    strings applied with probability p.  Averaging the oracle's Pauli-inserted
    states over all 16 draws must give the maximally mixed state I/4."""
    rng = np.random.default_rng(12)
    psi = ref.simulate(2, wc.random_gate_list(2, 10, rng, max_k=2), "0")
    rho = np.zeros((4, 4), dtype=complex)
    for code in range(16):
        a, b = wc.PAULI_LABELS[code // 4], wc.PAULI_LABELS[code % 4]
        factors = tuple(f for f in ((1, a), (0, b)) if f[1] != "I")
        v = ref.pauli_apply(psi, factors)
        rho += np.outer(v, v.conj()) / 16
    assert np.max(np.abs(rho - np.eye(4) / 4)) < 1e-15
    # p = 0 draws no Pauli and leaves the noiseless circuit
    noisy = wc.trajectory_batch(count=6, root_seed=11, p=0.3, n_range=(4, 7), depth_range=(3, 6))
    clean = wc.trajectory_batch(count=6, root_seed=11, p=0.0, n_range=(4, 7), depth_range=(3, 6))
    assert sum(t.n_inserted for t in noisy) > 0
    for a, b in zip(noisy, clean):
        assert (a.n, a.depth) == (b.n, b.depth)
        assert b.n_inserted == 0
        assert [g for g in a.gates if g.name not in ("X", "Y", "Z")] == b.gates
    # <Z_0> on basis states
    assert abs(ref.z0(ref.basis_state(5, 0)) - 1) < 1e-15
    assert abs(ref.z0(ref.basis_state(5, 1)) + 1) < 1e-15



def check_metrics():
    """The parity metrics against values fixed by mathematics.
    * RY(t)|0> = cos(t/2)|0> + sin(t/2)|1>, so against |0> the fidelity is
      cos^2(t/2) and 1-F = sin^2(t/2); on n qubits, |+>^n against |0..0> has
      fidelity 2^-n.
    * 1-F is blind to a global phase and to the scale of either state; the raw
      error |1 - |<ref|psi>|^2| of a scaled unit state c psi is |1 - c^2|.
    * Orthogonal states have 1-F = 1.
    * max-abs is the largest complex modulus of the difference."""
    zero = ref.basis_state(1, 0)
    for t in (0.0, 0.3, 1.1, math.pi / 2, 2.5, math.pi):
        psi = zero.copy()
        ref.apply(psi, ref.gate_matrix("RY", (t,)), (0,))
        want = math.sin(t / 2) ** 2
        assert abs(ref.fidelity_error(zero, psi) - want) < 1e-15, (t, ref.fidelity_error(zero, psi), want)
        assert abs(ref.fidelity_error(psi, zero) - want) < 1e-15
        assert abs(ref.fidelity_error_raw(zero, psi) - want) < 1e-15
        # a scaled copy: the normalised error is unchanged, the raw one is not
        assert abs(ref.fidelity_error(zero, 3.0 * psi) - want) < 1e-14
        assert abs(ref.fidelity_error(0.25 * zero, psi) - want) < 1e-14
    for n in range(1, 7):
        plus = ref.product_state(n, "+")
        z = ref.basis_state(n, 0)
        assert abs(ref.fidelity_error(z, plus) - (1 - 2.0 ** -n)) < 1e-15, n
    rng = np.random.default_rng(13)
    v = rng.normal(size=64) + 1j * rng.normal(size=64)
    v /= np.linalg.norm(v)
    for c, phi in ((1.0, 0.7), (0.5, -2.0), (1.0 + 1e-4, 3.0)):
        w = c * np.exp(1j * phi) * v
        assert abs(ref.fidelity_error(v, w)) < 1e-14, (c, phi)
        assert abs(ref.fidelity_error_raw(v, w) - abs(1 - c * c)) < 1e-13, (c, phi)
    # orthogonal states
    a = ref.product_state(3, "+")
    b = ref.product_state(3, "+-+")
    assert abs(ref.fidelity_error(a, b) - 1.0) < 1e-15
    assert abs(ref.fidelity_error_raw(a, b) - 1.0) < 1e-15
    # max-abs on hand-built vectors: moduli of complex differences
    r = np.array([1.0, 0.0, 0.5j, -0.25], dtype=complex)
    p = np.array([1.0, 3e-3 + 4e-3j, 0.5j, -0.25 + 1e-3], dtype=complex)
    assert abs(ref.max_abs(r, p) - 5e-3) < 1e-17
    assert abs(ref.max_abs(r, p.astype(np.complex64)) - 5e-3) < 1e-9
    assert ref.max_abs(r, r) == 0.0
    assert abs(ref.max_abs(r, -r) - 2.0) < 1e-16

ALL_CHECKS = [
    check_metrics,
    check_grover_worked_example,
    check_compress_worked_example,
    check_apply_vs_brute,
    check_large_k_vs_brute,
    check_ghz,
    check_qft_basis_states,
    check_gate_table,
    check_product_states,
    check_norm_and_reversibility,
    check_fusion_product,
    check_expectation,
    check_gradients,
    check_trajectories,
]
