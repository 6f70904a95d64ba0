"""Host side of the density-matrix path (no GPU): the library's super-operator
matrices (sv_super_op_matrix), applied as gates on the row-major vectorisation
by the oracle's gate application, agree with the oracle's channel
application, and malformed operators are refused."""
import numpy as np
import pytest

import paper_2111_06868_amd as sv
from oracle import density as dm
from oracle import ref
from workloads import circuits as wc


def _rand_rho(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    rho = a @ a.conj().T
    return rho / np.trace(rho)


def _lib_apply(rho, op):
    """rho -> the library's super-operator matrix as a gate on (q + n, q)."""
    n = rho.shape[0].bit_length() - 1
    v = rho.ravel().copy()
    ref.apply(v, op.matrix(), [q + n for q in op.qubits] + list(op.qubits))
    return v.reshape(rho.shape)


@pytest.mark.parametrize("qs,m", [((1,), 2), ((3, 0), 3), ((2, 0, 3), 2)])
def test_kraus_super_op_matrix_vs_oracle(qs, m):
    rho = _rand_rho(4, 1)
    K = wc.random_kraus_from_seed(10 + m, len(qs), m)
    got = _lib_apply(rho, sv.SuperOp(qs, left=K))
    want = dm.apply_op(rho, {"qubits": qs, "left": K})
    assert np.abs(got - want).max() < 1e-14


def test_general_s_form_and_matrix_form_vs_oracle():
    rho = _rand_rho(3, 2)
    L = wc.random_kraus_from_seed(5, 2, 3)
    R = wc.random_kraus_from_seed(6, 2, 2)
    s = np.array([[0.3, 0.1j], [0.2, -0.4], [0.05, 0.5]])
    op = sv.SuperOp((2, 0), left=L, right=R, s=s)
    want = dm.apply_op(rho, {"qubits": (2, 0), "left": L, "right": R, "s": s})
    assert np.abs(_lib_apply(rho, op) - want).max() < 1e-14
    S = op.matrix()
    assert np.abs(_lib_apply(rho, sv.SuperOp((2, 0), superop=S)) - want).max() < 1e-14


def test_channel_helpers_vs_oracle():
    rho = _rand_rho(3, 3)
    pairs = [(sv.depolarizing((0, 2), 0.2), dm.depolarizing((0, 2), 0.2)),
             (sv.depolarizing((1,), 0.7), dm.depolarizing((1,), 0.7)),
             (sv.dephasing(2, 0.3, "X"), dm.dephasing(2, 0.3, "X")),
             (sv.amplitude_damping(1, 0.45), dm.amplitude_damping(1, 0.45)),
             (sv.amplitude_damping(0, 0.3, 0.12), dm.amplitude_damping(0, 0.3, 0.12)),
             (sv.depolarizing((2, 1, 0), 0.35), dm.depolarizing((2, 1, 0), 0.35))]
    for lib_op, or_op in pairs:
        assert np.abs(_lib_apply(rho, lib_op) - dm.apply_op(rho, or_op)).max() < 1e-14
        # the constructors' own operators, applied by the oracle
        assert np.abs(dm.apply_op(rho, {"qubits": lib_op.qubits, "left": list(lib_op.left)})
                      - dm.apply_op(rho, or_op)).max() < 1e-14


def _psd(dim, rank, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((dim, rank)) + 1j * rng.standard_normal((dim, rank))
    s = a @ a.conj().T
    return s / np.trace(s).real


@pytest.mark.parametrize("qs,rank", [((0,), 4), ((2,), 1), ((1, 0), 16), ((0, 2), 5), ((2, 0, 1), 7)])
def test_pauli_channel_and_its_kraus_form_vs_oracle(qs, rank):
    rho = _rand_rho(3, 4)
    s = _psd(4 ** len(qs), rank, 30 + rank)
    want = dm.apply_op(rho, dm.pauli_channel(qs, s))
    op = sv.pauli_channel(qs, s)
    assert np.abs(_lib_apply(rho, op) - want).max() < 1e-14
    kf = sv.kraus_form(op)
    assert len(kf.left) == rank and kf.s is None
    assert np.abs(dm.apply_op(rho, {"qubits": qs, "left": list(kf.left)}) - want).max() < 1e-13
    assert np.abs(_lib_apply(rho, kf) - want).max() < 1e-13


def test_local_channels_are_one_channel_per_qubit():
    rho = _rand_rho(3, 5)
    ops = sv.local_channels(sv.amplitude_damping, (0, 2, 1), [0.1, 0.2, 0.3], 0.05)
    assert [o.qubits for o in ops] == [(0,), (2,), (1,)]
    want = rho
    for q, g in zip((0, 2, 1), (0.1, 0.2, 0.3)):
        want = dm.apply_op(want, dm.amplitude_damping(q, g, 0.05))
    got = rho
    for o in ops:
        got = _lib_apply(got, o)
    assert np.abs(got - want).max() < 1e-14


def test_channel_constructors_refuse_bad_input():
    with pytest.raises(ValueError):
        sv.depolarizing((0,), 1.5)
    with pytest.raises(ValueError):
        sv.depolarizing((0, 0), 0.1)
    with pytest.raises(ValueError):
        sv.amplitude_damping(0, 0.2, -0.1)
    with pytest.raises(ValueError):
        sv.dephasing(0, 0.2, "W")
    not_herm = np.zeros((4, 4), dtype=complex)
    not_herm[0, 1] = 1.0
    with pytest.raises(ValueError):
        sv.kraus_form(sv.pauli_channel((0,), not_herm))
    with pytest.raises(ValueError):
        sv.kraus_form(sv.pauli_channel((0,), np.diag([1.0, -0.5, 0, 0])))


def test_malformed_super_ops_are_refused():
    K = wc.random_kraus_from_seed(1, 1, 2)
    with pytest.raises(ValueError):
        sv.SuperOp((0, 1, 2, 3), left=wc.random_kraus_from_seed(1, 4, 1)).matrix()  # k = 4
    # the library's own checks, on a hand-made descriptor
    import ctypes
    from paper_2111_06868_amd import _native as N
    c, keep = N.sv_super_op(), []
    sv.SuperOp((0,), left=K).fill(c, keep)
    out = np.zeros(2 * 16, dtype=np.float64)
    optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert N.lib().sv_super_op_matrix(ctypes.byref(c), optr) == 0
    for field, value in (("k", 4), ("reserved", 1), ("n_left", 0), ("n_right", 65)):
        saved = getattr(c, field)
        setattr(c, field, value)
        assert N.lib().sv_super_op_matrix(ctypes.byref(c), optr) == -1, field
        setattr(c, field, saved)
    with pytest.raises(sv.SvError):
        sv.SuperOp((0,), left=K, right=K[:1]).matrix()  # s = identity needs equal counts
    bad = [k.copy() for k in K]
    bad[0][0, 0] = np.nan
    with pytest.raises(sv.SvError):
        sv.SuperOp((0,), left=bad).matrix()
