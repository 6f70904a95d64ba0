"""GPU parity of density-matrix evolution (sv_dm_run, sv_dm_expectation)
against the density-matrix oracle on the same seeded inputs, and the exact
noisy <Z_0> against the mean of sampled Pauli trajectories (paper,
Simulations with noise section: both treatments of the same channel).
Complex64 entries must match to 2e-5 (each entry of rho is at most 1 in
magnitude; the error is FP32 rounding accumulated over the circuit's blocks),
complex128 to 1e-12."""
import math
import sys

import numpy as np
import pytest

import paper_2111_06868_amd as sv
from oracle import density as dm
from oracle import ref
from workloads import circuits as wc
from helpers import to_binding

pytestmark = pytest.mark.gpu

TOL = {sv.PREC_FP32: 2e-5, sv.PREC_SPLIT_BF16: 2e-5, sv.PREC_SPLIT_BF16X3: 2e-5, sv.PREC_FP64: 1e-12}
TILE_FAMILY = {sv.PREC_FP32: "tile", sv.PREC_SPLIT_BF16: "tile_bf16", sv.PREC_SPLIT_BF16X3: "tile_bf16x3"}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield
    torch.cuda.synchronize()


def _noisy_case(rows, cols, depth, seed, p=0.02):
    """Gates plus matched operator lists: the library's SuperOp objects and
    the oracle's dicts (same inputs, built independently on each side)."""
    gates = wc.grid_rqc(rows, cols, depth, seed)
    n = rows * cols
    lib_ops, or_ops = [], []
    fs = [i for i, g in enumerate(gates) if g.name == "FSIM"]
    for i in fs:
        q = gates[i].qubits
        lib_ops.append(sv.depolarizing(q, p, after=i + 1))
        or_ops.append(dm.depolarizing(q, p, after=i + 1))
    mid = len(gates) // 2
    # amplitude damping, a random 2-qubit Kraus channel, a general s form and
    # a matrix super operator, all in the middle of the circuit
    lib_ops.append(sv.amplitude_damping(0, 0.1, after=mid))
    or_ops.append(dm.amplitude_damping(0, 0.1, after=mid))
    K = wc.random_kraus_from_seed(seed + 1, 2, 3)
    qk = (n - 1, 0)
    lib_ops.append(sv.SuperOp(qk, left=K, after=mid))
    or_ops.append({"qubits": qk, "left": K, "after": mid})
    L = wc.random_kraus_from_seed(seed + 2, 1, 2)
    s = np.array([[0.9, 0.05j], [-0.05j, 0.1]])
    lib_ops.append(sv.SuperOp((1,), left=L, right=L, s=s, after=mid))
    or_ops.append({"qubits": (1,), "left": L, "right": L, "s": s, "after": mid})
    S = sv.amplitude_damping(0, 0.3).matrix()
    lib_ops.append(sv.SuperOp((n - 1,), superop=S, after=mid))
    or_ops.append({"qubits": (n - 1,), "superop": S, "after": mid})
    key = lambda o: o.after if hasattr(o, "after") else o["after"]
    lib_ops.sort(key=key)
    or_ops.sort(key=key)
    return n, gates, lib_ops, or_ops


def _check(tag, want, got, tol):
    err = float(np.abs(want - got).max())
    print("[parity] %-44s max_abs=%.3e" % (tag, err), flush=True)
    sys.stdout.flush()
    assert err <= tol, "%s: max_abs %.3e > %.1e" % (tag, err, tol)


@pytest.mark.parametrize("rule,max_k", [(sv.RULE_NONE, 6), (sv.RULE_PAPER, 4), (sv.RULE_ENHANCED, 6),
                                        (sv.RULE_ENHANCED, 5)])
@pytest.mark.parametrize("dtype,prec", [("c64", sv.PREC_FP32), ("c64", sv.PREC_SPLIT_BF16), ("c128", sv.PREC_FP64)])
def test_dm_small_vs_oracle(rule, max_k, dtype, prec):
    n, gates, lib_ops, or_ops = _noisy_case(2, 2, 6, seed=21)
    want = dm.simulate(n, gates, or_ops)
    rho = sv.DensityMatrix(n, dtype).run(to_binding(gates), lib_ops, max_k=max_k, precision=prec, rule=rule)
    _check("dm n=%d %s prec=%d rule=%d k<=%d" % (n, dtype, prec, rule, max_k), want, rho.read(), TOL[prec])


@pytest.mark.parametrize("prec", [sv.PREC_FP32, sv.PREC_SPLIT_BF16, sv.PREC_SPLIT_BF16X3])
def test_dm_tile_passes_vs_oracle(prec):
    # 7 qubits: rho is a 14-qubit state, so the tiled rule runs LDS tile passes
    n, gates, lib_ops, or_ops = _noisy_case(1, 7, 5, seed=5)
    want = dm.simulate(n, gates, or_ops)
    sv.stats_reset()
    sv.stats_enable(True)
    rho = sv.DensityMatrix(n, "c64").run(to_binding(gates), lib_ops, max_k=4, precision=prec,
                                         rule=sv.RULE_TILED)
    got = rho.read()
    sv.stats_enable(False)
    tiles = sum(sv.stats_query(TILE_FAMILY[prec], k)[0] for k in range(1, 17))
    assert tiles > 0, "no tile pass ran"
    _check("dm n=%d tiled prec=%d (%d tile launches)" % (n, prec, tiles), want, got, TOL[prec])


@pytest.mark.parametrize("dtype,prec", [("c64", sv.PREC_FP32), ("c128", sv.PREC_FP64)])
def test_dm_expectation_vs_oracle(dtype, prec):
    n, gates, lib_ops, or_ops = _noisy_case(2, 3, 5, seed=8)
    want_rho = dm.simulate(n, gates, or_ops)
    rho = sv.DensityMatrix(n, dtype).run(to_binding(gates), lib_ops, max_k=4, precision=prec,
                                         rule=sv.RULE_ENHANCED)
    terms = ([(1.0, ((i, "Z"), (i + 1, "Z"))) for i in range(n - 1)]
             + [(0.5, ((i, "X"),)) for i in range(n)]
             + [(0.3, ((0, "Y"), (2, "Y"))), (-0.7, ((1, "X"), (4, "Y"), (5, "Z"))), (0.25, ())])
    want = dm.expectation(want_rho, terms)
    got = rho.expectation(terms)
    tol = 1e-5 if dtype == "c64" else 1e-12
    print("[parity] dm Tr(rho H) %s: %.12f vs %.12f" % (dtype, got, want), flush=True)
    assert abs(got - want) <= tol
    assert abs(rho.trace() - np.trace(want_rho).real) <= tol


def test_dm_refuses_fp16_and_odd_states():
    rho = sv.DensityMatrix(2, "c64")
    with pytest.raises(sv.SvError):
        rho.run([("H", (0,))], [], precision=sv.PREC_SPLIT_FP16)
    odd = sv.DensityMatrix(2, "c64")
    odd.state = sv.State(5, "c64")
    with pytest.raises(sv.SvError):
        odd.run([("H", (0,))])
    with pytest.raises(sv.SvError):
        odd.expectation([(1.0, ((0, "Z"),))])
    with pytest.raises(sv.SvError):  # a gate on qubit 2 of a 2-qubit rho
        rho.run([("H", (2,))])
    with pytest.raises(sv.SvError):  # a 2-qubit channel is a 4-qubit gate: max_k 3 is too small
        rho.run([("H", (0,))], [sv.depolarizing((0, 1), 0.1, after=1)], max_k=3, rule=sv.RULE_ENHANCED)
    with pytest.raises(sv.SvError):  # operators out of order
        rho.run([("H", (0,)), ("H", (1,))], [sv.amplitude_damping(0, 0.1, after=2),
                                              sv.amplitude_damping(0, 0.1, after=1)])


def test_dm_exact_z0_matches_trajectory_mean():
    # the same depolarizing channel, evolved exactly and sampled on pure
    # states: the sample mean of <Z_0> must agree within 5 standard errors
    p = 0.05
    gates = wc.grid_rqc(2, 4, 10, seed=13)
    n = 8
    ops = [sv.depolarizing(g.qubits, p, after=i + 1) for i, g in enumerate(gates) if g.name == "FSIM"]
    rho = sv.DensityMatrix(n, "c128").run(to_binding(gates), ops, max_k=4, rule=sv.RULE_ENHANCED)
    exact = rho.expectation([(1.0, ((0, "Z"),))])
    trajs = wc.pauli_trajectories(gates, p, 2048, seed=77)
    z = sv.Batch([(n, to_binding(t)) for t in trajs], max_k=4).run()
    mean, se = float(np.mean(z)), float(np.std(z) / math.sqrt(len(z)))
    print("[parity] exact <Z0> %.6f, trajectory mean %.6f +- %.6f" % (exact, mean, se), flush=True)
    assert abs(mean - exact) <= 5 * se + 1e-6


# ------------------------------------------------ Kraus channels sampled on states
def _random_state(n, dtype, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi /= np.linalg.norm(psi)
    return psi, sv.State(n, dtype).write(psi)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("qs,m", [((0,), 2), ((11,), 4), ((3, 9), 3), ((5, 0), 4), ((10, 2, 6), 5),
                                  ((1, 0, 11), 16)])
def test_kraus_probabilities_vs_oracle(dtype, qs, m):
    n = 12
    psi, st = _random_state(n, dtype, seed=len(qs) * 10 + m)
    K = wc.random_kraus_from_seed(100 + m, len(qs), m)
    got = st.kraus_probabilities(sv.SuperOp(qs, left=K))
    want = np.array(dm.kraus_probabilities(psi, K, qs))
    rel = float(np.abs(got - want).max() / want.max())
    print("[parity] Kraus weights %s q=%s m=%d: rel %.3e" % (dtype, qs, m, rel), flush=True)
    assert rel <= (1e-6 if dtype == "c64" else 1e-12)
    assert abs(got.sum() - 1.0) <= (1e-6 if dtype == "c64" else 1e-12)


def _jump_case(n, seed, count):
    gates = wc.grid_rqc(2, n // 2, 6, seed)
    rng = np.random.default_rng(seed)
    lib_ops, or_ops = [], []
    for i, g in enumerate(gates):
        if g.name == "FSIM" and rng.random() < 0.5:
            q = int(rng.integers(n))
            lib_ops.append(sv.amplitude_damping(q, 0.2, after=i + 1))
            or_ops.append(dm.amplitude_damping(q, 0.2, after=i + 1))
        if len(lib_ops) >= count:
            break
    K = wc.random_kraus_from_seed(seed, 2, 3)
    last = lib_ops[-1].after
    lib_ops.append(sv.SuperOp((1, n - 1), left=K, after=last))
    or_ops.append({"qubits": (1, n - 1), "left": K, "after": last})
    return gates, lib_ops, or_ops


@pytest.mark.parametrize("dtype,prec", [("c64", sv.PREC_FP32), ("c128", sv.PREC_FP64)])
def test_trajectory_vs_oracle(dtype, prec):
    n = 10
    gates, lib_ops, or_ops = _jump_case(n, seed=3, count=8)
    u = np.random.default_rng(5).random(len(lib_ops))
    u[::2] = 0.96 + 0.03 * u[::2]  # high draws on every other channel force jumps
    st = sv.State(n, dtype)
    got = st.run_trajectory(to_binding(gates), lib_ops, u, max_k=4, precision=prec, rule=sv.RULE_ENHANCED)
    want_psi, want = dm.trajectory(n, gates, or_ops, u)
    print("[parity] trajectory %s outcomes %s" % (dtype, [int(x) for x in got]), flush=True)
    assert [int(x) for x in got] == list(want)
    assert any(x > 0 for x in want), "no jump in the case"
    psi = st.read().astype(np.complex128)
    err = float(np.abs(psi - want_psi).max())
    print("[parity] trajectory %s max_abs %.3e" % (dtype, err), flush=True)
    assert err <= (2e-6 if dtype == "c64" else 1e-12)


def test_jump_trajectory_mean_matches_density_matrix():
    # amplitude damping sampled on pure states against the exact density matrix
    n = 8
    gates, lib_ops, _ = _jump_case(n, seed=9, count=10)
    exact = sv.DensityMatrix(n, "c128").run(to_binding(gates), lib_ops, max_k=4,
                                            rule=sv.RULE_ENHANCED).expectation([(1.0, ((0, "Z"),))])
    rng = np.random.default_rng(17)
    ga = sv.GateArray(to_binding(gates))
    st = sv.State(n, "c64")
    Z0 = sv.pauli_sum([(1.0, ((0, "Z"),))])
    z = []
    for _ in range(400):
        st.set_basis(0)
        st.run_trajectory(ga, lib_ops, rng.random(len(lib_ops)), max_k=4, rule=sv.RULE_ENHANCED)
        z.append(st.expectation(Z0))
    mean, se = float(np.mean(z)), float(np.std(z) / math.sqrt(len(z)))
    print("[parity] exact <Z0> %.6f, jump-trajectory mean %.6f +- %.6f" % (exact, mean, se), flush=True)
    assert abs(mean - exact) <= 5 * se + 1e-6


def test_density_and_sampling_edge_cases():
    # one-qubit rho: operators only (no gates), one before the first gate
    rho = sv.DensityMatrix(1, "c128").run([], [sv.amplitude_damping(0, 0.5, after=0)])
    assert np.abs(rho.read() - np.diag([1.0, 0.0])).max() < 1e-15
    rho = sv.DensityMatrix(1, "c128")
    rho.run([("X", (0,))], [sv.dephasing(0, 0.3, after=0), sv.amplitude_damping(0, 0.25, after=1)])
    assert np.abs(rho.read() - np.diag([0.25, 0.75])).max() < 1e-15
    assert abs(rho.trace() - 1.0) < 1e-15
    # |index><index|
    assert abs(sv.DensityMatrix(3, "c128").set_basis(5).expectation([(1.0, ((0, "Z"),))]) + 1.0) < 1e-15
    # a trajectory without operators is the plain run
    gates = to_binding(wc.grid_rqc(2, 3, 4, seed=2))
    a = sv.State(6, "c128").run(gates, max_k=4, rule=sv.RULE_ENHANCED).read()
    st = sv.State(6, "c128")
    assert len(st.run_trajectory(gates, [], [], max_k=4, rule=sv.RULE_ENHANCED)) == 0
    assert np.abs(st.read() - a).max() < 1e-15
    # measuring every qubit of a basis state is deterministic, whatever the draws
    st = sv.State(5, "c64").set_basis(0b10110)
    bits, p = st.measure([4, 3, 2, 1, 0], [0.99, 0.01, 0.5, 0.99, 0.01])
    assert bits == "10110" and abs(p - 1.0) < 1e-12
    # a projection with probability 0 cannot be renormalised
    with pytest.raises(sv.SvError):
        sv.State(2, "c64").project((0,), "1", renormalize=True)


@pytest.mark.parametrize("prec", [sv.PREC_SPLIT_BF16, sv.PREC_SPLIT_BF16X3])
def test_dm_many_tiles_vs_oracle(prec):
    # 9 qubits: rho is an 18-qubit state, 16 tiles of 2^14 per tile pass
    n, gates, lib_ops, or_ops = _noisy_case(3, 3, 4, seed=31)
    want = dm.simulate(n, gates, or_ops)
    sv.stats_reset()
    sv.stats_enable(True)
    rho = sv.DensityMatrix(n, "c64").run(to_binding(gates), lib_ops, max_k=4, precision=prec,
                                         rule=sv.RULE_TILED)
    got = rho.read()
    tr = rho.trace()
    sv.stats_enable(False)
    tiles = sum(sv.stats_query(TILE_FAMILY[prec], k)[0] for k in range(1, 17))
    assert tiles > 0
    _check("dm n=%d tiled prec=%d, 16 tiles (%d launches), trace error %.2e" % (n, prec, tiles,
                                                                             tr - np.trace(want).real),
           want, got, TOL[prec])
    if prec == sv.PREC_SPLIT_BF16X3:  # FP32's accuracy (the case holds non-trace-preserving operators)
        assert abs(tr - np.trace(want).real) <= 1e-6 and float(np.abs(got - want).max()) <= 1e-7


@pytest.mark.parametrize("prec", [sv.PREC_FP32, sv.PREC_SPLIT_BF16, sv.PREC_SPLIT_BF16X3])
def test_trajectory_with_tile_passes_vs_oracle(prec):
    # 16 qubits: the gate runs between channels go through tile passes
    n = 16
    gates, lib_ops, or_ops = _jump_case(n, seed=21, count=6)
    u = np.random.default_rng(8).random(len(lib_ops))
    u[1::2] = 0.95 + 0.04 * u[1::2]
    st = sv.State(n, "c64")
    sv.stats_reset()
    sv.stats_enable(True)
    got = st.run_trajectory(to_binding(gates), lib_ops, u, max_k=4, precision=prec, rule=sv.RULE_TILED)
    psi = st.read().astype(np.complex128)
    sv.stats_enable(False)
    assert sum(sv.stats_query(TILE_FAMILY[prec], k)[0] for k in range(1, 17)) > 0, "no tile pass ran"
    want_psi, want = dm.trajectory(n, gates, or_ops, u)
    assert [int(x) for x in got] == list(want) and any(x > 0 for x in want)
    fe = 1 - abs(np.vdot(want_psi, psi)) ** 2 / (np.vdot(psi, psi).real * np.vdot(want_psi, want_psi).real)
    print("[parity] tiled trajectory n=%d prec=%d outcomes %s 1-F %.3e" % (n, prec, list(want), fe), flush=True)
    assert fe <= 1e-5


def test_kraus_probabilities_beyond_16_operators():
    # 40 operators on 3 qubits: three launches of the weights kernel
    for dtype, tol in (("c64", 1e-6), ("c128", 1e-12)):
        n = 12
        psi, st = _random_state(n, dtype, seed=41)
        K = wc.random_kraus_from_seed(140, 3, 40)
        got = st.kraus_probabilities(sv.SuperOp((4, 0, 9), left=K))
        want = np.array(dm.kraus_probabilities(psi, K, (4, 0, 9)))
        rel = float(np.abs(got - want).max() / want.max())
        print("[parity] Kraus weights %s, 40 operators: rel %.3e" % (dtype, rel), flush=True)
        assert got.size == 40 and rel <= tol


def _psd(dim, rank, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((dim, rank)) + 1j * rng.standard_normal((dim, rank))
    s = a @ a.conj().T
    return s / np.trace(s).real


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_sampled_general_pauli_channel_branches_vs_density_oracle(dtype):
    """A GlobalPauliChannel with a general (rank-3, off-diagonal) s and a
    generalized amplitude damping, sampled on pure states on the GPU: every
    outcome branch, drawn with the middle of its interval and weighted by its
    probability, sums to the density-matrix oracle's rho."""
    n = 5
    gates = wc.grid_rqc(1, 5, 4, seed=21)
    # a trace-preserving s of rank 3: s_ij = sum_m c_mi conj(c_mj), c_m the Pauli
    # coefficients of three random Kraus operators (sum_m K_m^dagger K_m = I)
    P = [dm.pauli_string(a + b) for a in "IXYZ" for b in "IXYZ"]
    C = np.array([[np.trace(Pi.conj().T @ K) / 4 for Pi in P] for K in wc.random_kraus_from_seed(22, 2, 3)])
    s = C.T @ C.conj()
    mid = len(gates) // 2
    lib_ops = [sv.pauli_channel((3, 1), s, after=mid), sv.amplitude_damping(2, 0.3, 0.1, after=len(gates))]
    or_ops = [dm.pauli_channel((3, 1), s, after=mid), dm.amplitude_damping(2, 0.3, 0.1, after=len(gates))]
    want = dm.simulate(n, gates, or_ops)
    bound = to_binding(gates)
    acc = np.zeros_like(want)
    count = [0]

    def walk(psi, start, j, weight):
        stop = lib_ops[j].after if j < len(lib_ops) else len(gates)
        st = sv.State(n, dtype).write(psi)
        st.run(bound[start:stop], max_k=4, rule=sv.RULE_ENHANCED)
        if j == len(lib_ops):
            v = st.read().astype(np.complex128)
            acc[:] += weight * np.outer(v, v.conj())
            count[0] += 1
            return
        p = st.kraus_probabilities(lib_ops[j])
        total, run = p.sum(), 0.0
        before = st.read()
        for i, w in enumerate(p):
            if w > 1e-12:
                br = sv.State(n, dtype).write(before)
                pick, _ = br.apply_kraus_sampled(lib_ops[j], (run + w / 2) / total)
                assert pick == i
                walk(br.read(), stop, j + 1, weight * w / total)
            run += w

    walk(ref.product_state(n, "0"), 0, 0, 1.0)
    err = float(np.abs(acc - want).max())
    print("[parity] sampled Pauli channel (general s) branches %s: %d branches, max |d rho| %.3e"
          % (dtype, count[0], err), flush=True)
    assert count[0] == 3 * 3
    assert err <= (2e-6 if dtype == "c64" else 1e-12)


@pytest.mark.parametrize("dtype,prec", [("c64", sv.PREC_FP32), ("c128", sv.PREC_FP64)])
def test_dm_library_channels_vs_oracle(dtype, prec):
    """Density matrices with the library-built channels of the Noisy gates
    section: a general Pauli channel, its Kraus form, the generalized
    amplitude damping, a three-qubit depolarizing channel and local dephasing."""
    n = 4
    gates = wc.grid_rqc(2, 2, 5, seed=31)
    s = _psd(16, 5, 32)
    a, b = 4, len(gates) - 3
    lib_ops = [sv.pauli_channel((0, 3), s, after=a), sv.kraus_form(sv.pauli_channel((2, 1), s, after=a + 1)),
               sv.amplitude_damping(1, 0.2, 0.05, after=b), sv.depolarizing((3, 0, 2), 0.15, after=b)]
    lib_ops += sv.local_channels(sv.dephasing, (0, 1, 2), [0.1, 0.2, 0.3], "X", after=len(gates))
    or_ops = [dm.pauli_channel((0, 3), s, after=a), dm.pauli_channel((2, 1), s, after=a + 1),
              dm.amplitude_damping(1, 0.2, 0.05, after=b), dm.depolarizing((3, 0, 2), 0.15, after=b)]
    or_ops += [dm.dephasing(q, p, "X", after=len(gates)) for q, p in ((0, 0.1), (1, 0.2), (2, 0.3))]
    want = dm.simulate(n, gates, or_ops)
    rho = sv.DensityMatrix(n, dtype).run(to_binding(gates), lib_ops, max_k=6, rule=sv.RULE_ENHANCED, precision=prec)
    err = float(np.abs(rho.read() - want).max())
    print("[parity] density matrix with library channels %s: max %.3e" % (dtype, err), flush=True)
    assert err <= (1e-6 if dtype == "c64" else 1e-12)
