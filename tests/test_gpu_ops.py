"""GPU parity of projections, measurements and controlled gates (sv_project,
sv_measure, sv_controlled_gate) against oracle/ops.py on the same seeded
inputs, and the paper's Grover example as one fused diagonal gate."""
import os

import numpy as np
import pytest

import paper_2111_06868_amd as sv
from oracle import ops, ref
from workloads import circuits as wc
from helpers import to_binding

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield
    torch.cuda.synchronize()


def _state(n, dtype, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi /= np.linalg.norm(psi)
    return psi, sv.State(n, dtype).write(psi)


TOL = {"c64": 2e-6, "c128": 1e-12}


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("qs,bits,renorm", [((0,), "1", True), ((13,), "0", False), ((2, 9), "10", True),
                                            ((11, 1, 6), "011", True), ((5, 0, 12, 3, 8, 10), "110100", False)])
def test_project_vs_oracle(dtype, qs, bits, renorm):
    n = 14
    psi, st = _state(n, dtype, seed=len(qs))
    p = st.project(qs, bits, renorm)
    want, pw = ops.project(psi, qs, bits, renorm)
    err = float(np.abs(st.read().astype(np.complex128) - want).max())
    print("[parity] project %s q=%s bits=%s: p %.3e vs %.3e, max_abs %.3e" % (dtype, qs, bits, p, pw, err), flush=True)
    assert abs(p - pw) <= TOL[dtype] * max(pw, 1e-3)
    assert err <= TOL[dtype] * (1.0 if renorm else 0.1)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_measure_vs_oracle(dtype):
    n = 12
    psi, st = _state(n, dtype, seed=7)
    qs = (3, 11, 0, 7)
    u = [0.41, 0.93, 0.07, 0.66]
    bits, p = st.measure(qs, u)
    want, wbits, wp = ops.measure(psi, qs, u)
    err = float(np.abs(st.read().astype(np.complex128) - want).max())
    print("[parity] measure %s: %s (p %.4e) vs %s (p %.4e), max_abs %.3e" % (dtype, bits, p, wbits, wp, err),
          flush=True)
    assert bits == wbits
    assert abs(p - wp) <= TOL[dtype] * wp
    assert err <= TOL[dtype] * 10


@pytest.mark.parametrize("dtype,prec", [("c64", sv.PREC_FP32), ("c128", sv.PREC_FP64)])
def test_controlled_gates_in_a_circuit(dtype, prec):
    n = 8
    gates = wc.grid_rqc(2, 4, 3, seed=14)
    bound = to_binding(gates)
    extra = [sv.controlled(("X", (2,)), (0, 5)), sv.controlled(("FSIM", (3, 6), (0.4, 0.9)), (1,)),
             sv.controlled(("MATRIX", (7,), (), -1, wc.haar_unitary_from_seed(3, 1)), (4, 2, 6))]
    circ = bound[:10] + extra + bound[10:]
    oracle_ops = [(ref.matrix_of(g), g.qubits) for g in gates[:10]]
    oracle_ops += [(ops.controlled(ref.gate_matrix("X"), 2), (0, 5, 2)),
                   (ops.controlled(ref.gate_matrix("FSIM", (0.4, 0.9)), 1), (1, 3, 6)),
                   (ops.controlled(wc.haar_unitary_from_seed(3, 1), 3), (4, 2, 6, 7))]
    oracle_ops += [(ref.matrix_of(g), g.qubits) for g in gates[10:]]
    want = ref.run_matrices(ref.product_state(n, "0"), oracle_ops)
    for rule, k in [(sv.RULE_NONE, 6), (sv.RULE_ENHANCED, 5)]:
        got = sv.State(n, dtype).run(circ, max_k=k, precision=prec, rule=rule).read()
        fe = ref.fidelity_error(want, got)
        print("[parity] controlled gates %s rule=%d: 1-F %.3e" % (dtype, rule, fe), flush=True)
        assert fe <= (1e-5 if dtype == "c64" else 1e-12)
        assert ref.max_abs(want, got) <= (2e-6 if dtype == "c64" else 1e-12)


def test_grover_oracle_as_a_diagonal_gate_matches_the_paper():
    # order = [0, 1, 2]: the paper's qubits 1, 2 are positions 1, 0; the oracle
    # psi - 2 P00 psi is the diagonal gate diag(-1, 1, 1, 1) on them
    st = sv.State(3, "c128").set_product("+")
    st.apply_gate(("MATRIX", (1, 0), (), -1, np.diag([-1.0, 1.0, 1.0, 1.0])))
    got = st.read()
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "grover_3q.txt"))
            if l.strip() and not l.startswith("#")]
    for b, v in rows:
        assert abs(got[int(b, 2)].real - float(v)) < 5e-7
    # the same with sv_project: the projection on 00 has probability 1/4
    st2 = sv.State(3, "c128").set_product("+")
    assert abs(st2.project((1, 0), "00", renormalize=False) - 0.25) < 1e-15


def test_split_fp16_refuses_non_unitary_matrices():
    A = np.array([[1.0, 0.5], [0.0, 1.0]])  # not unitary: it can raise the norm
    U = wc.haar_unitary_from_seed(9, 1)
    st = sv.State(14, "c64")
    with pytest.raises(sv.SvError):
        st.run([("MATRIX", (3,), (), -1, A)], max_k=4, precision=sv.PREC_SPLIT_FP16, rule=sv.RULE_TILED)
    st.run([("MATRIX", (3,), (), -1, U)], max_k=4, precision=sv.PREC_SPLIT_FP16, rule=sv.RULE_TILED)
    plan = sv.fuse([("MATRIX", (3,), (), -1, A), ("H", (4,))], 14, 4, sv.RULE_TILED)
    with pytest.raises(sv.SvError):
        st.apply_plan(plan, precision=sv.PREC_SPLIT_FP16)
    st.apply_plan(plan, precision=sv.PREC_SPLIT_BF16)  # split BF16 keeps FP32's range
    with pytest.raises(sv.SvError):
        sv.Batch([(14, [("MATRIX", (0,), (), -1, A)])], max_k=4, precision=sv.PREC_SPLIT_FP16)
