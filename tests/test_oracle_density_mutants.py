"""Plant plausible mistakes in the density-matrix, sampling and projection
oracles (CPU only) and check that their pins catch each one: every mutant must
make at least one pin of tests/test_oracle_density.py or test_oracle_ops.py
fail."""
import numpy as np
import pytest

import test_oracle_density as D
import test_oracle_ops as O
from oracle import density as dm
from oracle import ops, ref

_apply_gate = dm.apply_gate
_apply_kraus = dm.apply_kraus_super
_apply_matrix = dm.apply_matrix_super
_depol = dm.depolarizing
_damp = dm.amplitude_damping
_pauli_ch = dm.pauli_channel
_sample = dm.sample_kraus
_project = ops.project
_measure = ops.measure
_controlled = ops.controlled

PINS = [
    D.test_pure_circuit_is_psi_psi_dagger,
    D.test_depolarizing_closed_forms,
    D.test_amplitude_damping_closed_form,
    lambda: D.test_dephasing_of_rotating_spin(0.7),
    D.test_channel_equals_exact_mixture_of_sampled_paulis,
    D.test_matrix_super_gate_matches_kraus_form,
    D.test_random_channel_keeps_a_density_matrix,
    D.test_sampled_amplitude_damping_closed_form,
    D.test_branches_of_sampled_channels_sum_to_the_density_matrix,
    D.test_trajectory_follows_the_drawn_branch,
    D.test_generalized_amplitude_damping_closed_forms,
    D.test_pauli_channel_closed_forms,
    O.test_grover_oracle_by_projection_matches_the_paper,
    O.test_controlled_gates_are_the_textbook_ones,
    O.test_measure_ghz_collapses,
    O.test_born_rule_by_brute_force,
]


def mut_right_transpose(mp):
    """U rho U^T instead of U rho U^dagger."""
    def f(rho, U, qubits):
        A = dm._left(rho, U, qubits)
        return dm._left(A.T.copy(), U, qubits).T.copy()
    mp.setattr(dm, "apply_gate", f)


def mut_kraus_ignores_s(mp):
    mp.setattr(dm, "apply_kraus_super", lambda rho, left, right, s, q: _apply_kraus(rho, left, right, None, q))


def mut_kraus_right_not_adjoint(mp):
    """L rho R instead of L rho R^dagger."""
    def f(rho, left, right, s, qubits):
        out = np.zeros_like(rho)
        for i, L in enumerate(left):
            A = dm._left(rho, L, qubits)
            for j, R in enumerate(right):
                w = (1.0 if i == j else 0.0) if s is None else s[i][j]
                if w:
                    out += w * dm._left(A.T.copy(), np.asarray(R).T, qubits).T
        return out
    mp.setattr(dm, "apply_kraus_super", f)


def mut_matrix_super_column_major(mp):
    """The MatrixSuperGate applied with the column index most significant."""
    def f(rho, S, qubits):
        n = rho.shape[0].bit_length() - 1
        v = rho.ravel().copy()
        ref.apply(v, S, list(qubits) + [q + n for q in qubits])
        return v.reshape(rho.shape)
    mp.setattr(dm, "apply_matrix_super", f)


def mut_depolarizing_weight(mp):
    """p/d instead of p/d^2 per Pauli string."""
    def f(qubits, p, after=0):
        op = _depol(qubits, p, after)
        d = 1 << len(qubits)
        op["left"] = [K * np.sqrt(d) if i else K for i, K in enumerate(op["left"])]
        return op
    mp.setattr(dm, "depolarizing", f)


def mut_damping_transposed(mp):
    def f(qubit, gamma, excitation=0.0, after=0):
        op = _damp(qubit, gamma, excitation, after)
        op["left"] = [op["left"][0], op["left"][1].T.copy()] + op["left"][2:]
        return op
    mp.setattr(dm, "amplitude_damping", f)


def mut_excitation_keeps_k0(mp):
    """The excitation operator added without shrinking |0><0| in K0."""
    def f(qubit, gamma, excitation=0.0, after=0):
        op = _damp(qubit, gamma, excitation, after)
        op["left"][0] = np.diag([1.0, np.sqrt(1 - gamma)]).astype(complex)
        return op
    mp.setattr(dm, "amplitude_damping", f)


def mut_excitation_swapped_rates(mp):
    """The excitation rate on the decay operator and the decay rate on the excitation one."""
    def f(qubit, gamma, excitation=0.0, after=0):
        op = _damp(qubit, gamma, excitation, after)
        if excitation > 0:
            op["left"][1], op["left"][2] = (np.sqrt(excitation / gamma) * op["left"][1],
                                            np.sqrt(gamma / excitation) * op["left"][2])
        return op
    mp.setattr(dm, "amplitude_damping", f)


def mut_pauli_channel_transposed_s(mp):
    """s_ji in place of s_ij."""
    mp.setattr(dm, "pauli_channel", lambda qubits, s, after=0: _pauli_ch(qubits, np.asarray(s).T, after))


def mut_pauli_channel_reversed_digits(mp):
    """The first base-4 digit on the last qubit."""
    mp.setattr(dm, "pauli_channel", lambda qubits, s, after=0: _pauli_ch(tuple(qubits)[::-1], s, after))


def mut_sample_last_outcome(mp):
    """The last outcome whose running sum exceeds u, instead of the first."""
    def f(psi, kraus, qubits, u):
        p = dm.kraus_probabilities(psi, kraus, qubits)
        total, run, pick = sum(p), 0.0, -1
        for i, w in enumerate(p):
            run += w
            if w > 0 and u * total < run:
                pick = i
        out = ref.apply(psi.copy(), kraus[pick], qubits) / np.sqrt(p[pick])
        return out, pick
    mp.setattr(dm, "sample_kraus", f)


def mut_sample_unnormalised(mp):
    def f(psi, kraus, qubits, u):
        out, pick = _sample(psi, kraus, qubits, u)
        p = dm.kraus_probabilities(psi, kraus, qubits)[pick]
        return out * np.sqrt(p), pick
    mp.setattr(dm, "sample_kraus", f)


def mut_project_bits_reversed(mp):
    mp.setattr(ops, "project", lambda psi, q, bits, renormalize=True: _project(psi, q, bits[::-1], renormalize))


def mut_measure_rule_inverted(mp):
    def f(psi, qubits, uniforms):
        return _measure(psi, qubits, [1.0 - u for u in uniforms])
    mp.setattr(ops, "measure", f)


def mut_controlled_top_block(mp):
    def f(U, n_c):
        d = U.shape[0]
        C = np.eye(d << n_c, dtype=np.complex128)
        C[:d, :d] = U
        return C
    mp.setattr(ops, "controlled", f)


MUTANTS = [mut_right_transpose, mut_kraus_ignores_s, mut_kraus_right_not_adjoint, mut_matrix_super_column_major,
           mut_depolarizing_weight, mut_damping_transposed, mut_excitation_keeps_k0, mut_excitation_swapped_rates,
           mut_pauli_channel_transposed_s, mut_pauli_channel_reversed_digits, mut_sample_last_outcome,
           mut_sample_unnormalised,
           mut_project_bits_reversed, mut_measure_rule_inverted, mut_controlled_top_block]


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda f: f.__name__)
def test_mutant_is_caught(mutant, monkeypatch):
    mutant(monkeypatch)
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            return
    pytest.fail("planted mistake %s passed every pin" % mutant.__name__)
