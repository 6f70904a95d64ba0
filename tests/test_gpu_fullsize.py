"""GPU parity at the full workload sizes.

* 30 qubits, in the launch configuration the benchmark times (tiled rule,
  k <= 4, split-FP16 tile passes), with split-BF16 and three-part split-BF16
  tile passes, and in the enhanced FP32 configuration (k <= 5): a 100-gate prefix of the 845-gate circuit against the CPU oracle on
  the whole 2^30-amplitude state, then the whole circuit against a complex128
  GPU run (fidelity, raw fidelity, norm, first 2^20 amplitudes).
* 32 qubits: the 632-gate circuit with k = 4..6 blocks in FP32 and in split
  BF16 / FP16 against a complex128 GPU run.
* 34 qubits: tile passes (split BF16, split FP16 and FP32) on a 12-qubit
  circuit spread over the positions, every amplitude of its support against
  the oracle.
* 20-qubit ansatz: the energy and all 480 adjoint gradients against the
  oracle's parameter-shift and finite-difference values (stored by
  tests/golden/make_full_size_golden.py), plus a direct oracle check on a few.
These need a large GPU (up to 128 GiB) and host memory (up to 24 GiB)."""
import math
import os

import numpy as np
import pytest

import paper_2111_06868_amd as sv
from oracle import ref
from workloads import circuits as wc
from helpers import to_binding

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# the benchmark's configuration (tiled, split FP16), the other tile
# arithmetics and the enhanced FP32 one:
# (rule, max_k, precision, bound on 1-F, on max-abs, on |norm - 1|)
CONFIGS = {
    "tiled_fp16_k4": (sv.RULE_TILED, 4, sv.PREC_SPLIT_FP16, 1e-10, 1e-8, 1e-6),
    "tiled_bf16_k4": (sv.RULE_TILED, 4, sv.PREC_SPLIT_BF16, 1e-5, 1e-6, 1e-6),
    "enhanced_fp32_k5": (sv.RULE_ENHANCED, 5, sv.PREC_FP32, 1e-5, 1e-6, 1e-6),
    "tiled_bf16x3_k4": (sv.RULE_TILED, 4, sv.PREC_SPLIT_BF16X3, 1e-10, 1e-8, 1e-6),
}


def _fe_dev(a, b):
    return sv.fidelity_error(a, b)


@pytest.fixture(scope="module")
def prefix30():
    n, gates = wc.config_circuit(1)
    prefix = gates[:100]
    want = ref.simulate(n, prefix, "0")
    yield n, prefix, want


@pytest.mark.parametrize("cfg", sorted(CONFIGS))
def test_30q_prefix_vs_oracle_full_state(prefix30, cfg):
    rule, k, prec, tol_fe, tol_abs, tol_norm = CONFIGS[cfg]
    n, prefix, want = prefix30
    st = sv.State(n, "c64").run(to_binding(prefix), max_k=k, rule=rule, precision=prec)
    got = st.read()
    nd = abs(st.norm2() - 1)
    st.free()
    del st
    fe = ref.fidelity_error(want, got)
    fr = ref.fidelity_error_raw(want, got)
    ma = ref.max_abs(want, got)
    print("[parity] 30q prefix(100 gates) %s vs oracle (all 2^30): 1-F=%.3e raw 1-F=%.3e max_abs=%.3e "
          "|norm-1|=%.2e" % (cfg, fe, fr, ma, nd), flush=True)
    # raw 1-F also carries the norm drift
    assert fe <= tol_fe and fr <= tol_fe + 2 * tol_norm and ma <= tol_abs and nd <= tol_norm


@pytest.fixture(scope="module")
def ref30():
    n, gates = wc.config_circuit(1)
    g = sv.GateArray(to_binding(gates))
    refst = sv.State(n, "c128").run(g)
    assert abs(refst.norm2() - 1) <= 1e-12
    yield n, g, refst
    refst.free()


@pytest.mark.parametrize("cfg", sorted(CONFIGS))
def test_30q_full_circuit_vs_c128(ref30, cfg):
    rule, k, prec, tol_fe, tol_abs, tol_norm = CONFIGS[cfg]
    n, g, refst = ref30
    fused = sv.State(n, "c64").run(g, max_k=k, rule=rule, precision=prec)
    fe = _fe_dev(refst, fused)
    ov = refst.inner(fused)
    fr = 1.0 - abs(ov) ** 2  # raw: no renormalisation (the reference has norm 1 to 1e-12)
    nd = abs(fused.norm2() - 1)
    a = refst.read(0, 1 << 20)
    b = fused.read(0, 1 << 20)
    ma = float(np.max(np.abs(a - b)))
    fused.free()
    print("[parity] 30q full %s vs GPU c128: 1-F=%.3e raw 1-F=%.3e max_abs(first 2^20)=%.3e |norm-1|=%.2e"
          % (cfg, fe, fr, ma, nd), flush=True)
    assert fe <= tol_fe and abs(fr) <= tol_fe + 2 * tol_norm
    assert ma <= tol_abs and nd <= tol_norm
    # Porter-Thomas sanity (not a pin): 2^n sum |psi|^4 ~ 2 for a deep random circuit
    p = np.abs(a) ** 2
    assert 1.0 < (1 << 20) * np.sum(p ** 2) / np.sum(p) ** 2 < 3.0


def test_34q_high_positions_64bit_indexing():
    """A 34-qubit complex64 state (128 GiB): gates on the top positions,
    checked on the amplitudes they must produce (64-bit index arithmetic)."""
    import torch
    torch.cuda.empty_cache()
    n = 34
    st = sv.State(n, "c64")
    st.run([("H", (33,)), ("CX", (33, 0)), ("CX", (0, 32)), ("RZ", (32,), (0.8,))])
    hi = (1 << 33) | (1 << 32) | 1
    a0 = st.read(0, 1)[0]
    a1 = st.read(hi, 1)[0]
    r = 1 / math.sqrt(2)
    assert abs(a0 - r * np.exp(-0.4j)) <= 1e-6
    assert abs(a1 - r * np.exp(0.4j)) <= 1e-6
    assert abs(st.norm2() - 1) <= 1e-6
    # a dense block across the top of the state through the MFMA path
    M = wc.haar_unitary_from_seed(9, 5)
    st.run([("MATRIX", (33, 31, 29, 2, 0), (), -1, M)], max_k=5, rule=sv.RULE_ENHANCED)
    assert abs(st.norm2() - 1) <= 1e-5
    st.free()
    del st
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,tol_fe,tol_abs,tol_norm", [
    (sv.PREC_SPLIT_BF16, 1e-7, 5e-5, 1e-4),
    (sv.PREC_SPLIT_BF16X3, 1e-10, 1e-6, 1e-5),
    (sv.PREC_SPLIT_FP16, 1e-10, 1e-6, 1e-5),
    (sv.PREC_FP32, 1e-10, 1e-6, 1e-5),
])
def test_34q_tile_passes_vs_oracle(precision, tol_fe, tol_abs, tol_norm):
    """Tile passes (the benchmark's launch configuration: tiled rule, k <= 4)
    on a 34-qubit complex64 state (128 GiB).  A 12-qubit random circuit is
    placed on positions spread from 0 to 33, so the result is a 12-qubit state
    times |0..0> on the other 22 positions: the oracle's 12-qubit result fixes
    every amplitude.  All 4096 amplitudes of the support are compared one by
    one, and the norm shows that nothing leaked outside it."""
    import torch
    torch.cuda.empty_cache()
    n = 34
    pos = (0, 3, 7, 12, 16, 19, 23, 26, 28, 30, 32, 33)
    m = len(pos)
    small = wc.random_gate_list(m, 160, np.random.default_rng(34), max_k=2)
    gates = [wc.Gate(g.name, tuple(pos[q] for q in g.qubits), g.params) for g in small]
    plan = sv.fuse(to_binding(gates), n, 4, sv.RULE_TILED).blocks(False)
    assert sum(1 for b in plan if b.tile_pass >= 0) >= 2 * len(set(b.tile_pass for b in plan if b.tile_pass >= 0))
    want = ref.simulate(m, small)
    st = sv.State(n, "c64")
    st.run(to_binding(gates), max_k=4, rule=sv.RULE_TILED, precision=precision)
    idx = [sum(((j >> b) & 1) << pos[b] for b in range(m)) for j in range(1 << m)]
    got = np.array([st.read(i, 1)[0] for i in idx], dtype=np.complex128)
    fe = ref.fidelity_error(want, got)
    ma = ref.max_abs(want, got)
    nd = abs(st.norm2() - 1)
    print("[parity] 34q tile passes precision=%d: 1-F=%.3e max_abs=%.3e |norm-1|=%.3e" % (precision, fe, ma, nd))
    assert fe <= tol_fe and ma <= tol_abs and nd <= tol_norm
    st.free()
    del st
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def ref32():
    n, gates = wc.config_circuit(2)
    g = sv.GateArray(to_binding(gates))
    refst = sv.State(n, "c128").run(g, max_k=6, rule=sv.RULE_ENHANCED)
    assert abs(refst.norm2() - 1) <= 1e-12
    yield n, g, refst
    refst.free()


@pytest.mark.parametrize("precision", [sv.PREC_FP32, sv.PREC_SPLIT_BF16, sv.PREC_SPLIT_FP16])
def test_32q_blocks_vs_c128(ref32, precision):
    n, g, refst = ref32
    st = sv.State(n, "c64").run(g, max_k=6, rule=sv.RULE_ENHANCED, precision=precision)
    fe = _fe_dev(refst, st)
    ma = float(np.max(np.abs(refst.read(0, 1 << 20) - st.read(0, 1 << 20))))
    print("[parity] 32q fused k<=6 precision=%d vs GPU c128: 1-F=%.3e max_abs(first 2^20)=%.3e"
          % (precision, fe, ma), flush=True)
    assert fe <= 1e-5
    assert ma <= 1e-6


def _ansatz_golden():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "ansatz20_gradients.txt"))
            if ln.strip() and not ln.startswith("#")]
    e = float(rows[0][1])
    ps = np.array([float(r[1]) for r in rows[1:]])
    fd = np.array([float(r[2]) for r in rows[1:]])
    assert [int(r[0]) for r in rows[1:]] == list(range(480))
    return e, ps, fd


def test_20q_ansatz_adjoint_all_gradients():
    n = 20
    gates, thetas = wc.ansatz_circuit(n, 12, seed=3)
    H = wc.ansatz_observable(n)
    e_ref, ps, fd = _ansatz_golden()
    psi = sv.State(n, "c64").run(to_binding(gates), max_k=4, rule=sv.RULE_ENHANCED)
    e = psi.expectation(H)
    scratch = sv.State(n, "c64")
    g = sv.backward(psi, scratch, to_binding(gates), H, len(thetas))
    rel_ps = np.linalg.norm(g - ps) / np.linalg.norm(ps)
    rel_fd = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    scale = 1e-2 * np.max(np.abs(ps))
    worst = float(np.max(np.abs(g - ps) / np.maximum(np.abs(ps), scale)))
    print("[parity] 20q ansatz E=%.8f (oracle %.8f); all 480 gradients: rel vs PS %.3e, vs FD(h=1e-3) %.3e, "
          "worst component %.3e" % (e, e_ref, rel_ps, rel_fd, worst), flush=True)
    assert abs(e - e_ref) <= 1e-5
    assert rel_ps <= 1e-4 and rel_fd <= 1e-4
    assert worst <= 1e-4
    # the stored values against the oracle itself on a few angles
    idx = [0, 21, 239, 479]
    assert np.abs(ref.param_shift_grad(n, gates, thetas, H, indices=idx) - ps[idx]).max() <= 1e-12
    # the adjoint pass consumed psi back to |0..0>
    assert abs(abs(psi.read(0, 1)[0]) - 1) <= 1e-4


@pytest.mark.parametrize("rule", [sv.RULE_TILED, sv.RULE_ENHANCED])
def test_20q_ansatz_adjoint_split_fp16(rule):
    """The 20-qubit ansatz with the forward run and the adjoint sweep's undone
    gate runs in split FP16 (per-tile scales on both states): E and all 480
    gradients against the stored oracle values, as in FP32."""
    n = 20
    gates, thetas = wc.ansatz_circuit(n, 12, seed=3)
    H = wc.ansatz_observable(n)
    e_ref, ps, fd = _ansatz_golden()
    prec = sv.PREC_SPLIT_FP16
    psi = sv.State(n, "c64").run(to_binding(gates), max_k=4, rule=rule, precision=prec)
    e = psi.expectation(H)
    scratch = sv.State(n, "c64")
    g = sv.backward(psi, scratch, to_binding(gates), H, len(thetas), precision=prec)
    rel_ps = np.linalg.norm(g - ps) / np.linalg.norm(ps)
    scale = 1e-2 * np.max(np.abs(ps))
    worst = float(np.max(np.abs(g - ps) / np.maximum(np.abs(ps), scale)))
    print("[parity] 20q ansatz split FP16 rule=%d E=%.8f (oracle %.8f); rel vs PS %.3e, worst component %.3e"
          % (rule, e, e_ref, rel_ps, worst), flush=True)
    assert abs(e - e_ref) <= 1e-5
    assert rel_ps <= 1e-4 and worst <= 1e-4
    assert abs(abs(psi.read(0, 1)[0]) - 1) <= 1e-4
    with pytest.raises(ValueError):
        sv.backward(sv.State(n, "c128"), sv.State(n, "c128"), to_binding(gates), H, len(thetas), precision=prec)


@pytest.mark.parametrize("precision", [sv.PREC_SPLIT_FP16, sv.PREC_SPLIT_BF16X3])
def test_32q_tiled_vs_c128(ref32, precision):
    """The 32-qubit grid circuit in the 32-qubit bench configuration: tiled
    rule, k <= 4, started from |0..0> in the first tile pass (split FP16) or
    filled (split BF16X3), against the complex128 run: fidelity, amplitudes
    and norm (split FP16 keeps the complex64 norm for unitary blocks)."""
    n, g, refst = ref32
    st = sv.State(n, "c64").set_product("+")
    st.run(g, max_k=4, rule=sv.RULE_TILED, precision=precision, basis=0)
    fe = _fe_dev(refst, st)
    ma = float(np.max(np.abs(refst.read(0, 1 << 20) - st.read(0, 1 << 20))))
    nd = abs(st.norm2() - 1)
    print("[parity] 32q tiled k<=4 precision=%d vs GPU c128: 1-F=%.3e max_abs(first 2^20)=%.3e |norm-1|=%.2e"
          % (precision, fe, ma, nd), flush=True)
    assert fe <= 1e-10 and ma <= 1e-8 and nd <= 1e-6
    st.free()
