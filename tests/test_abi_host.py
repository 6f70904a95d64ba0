"""The C ABI library on the host (no GPU needed): it loads, exports every
declared symbol, and its host-only logic (gate table, fusion, argument
validation) agrees with the oracle.  No call here launches device work."""
import ctypes
import math

import numpy as np
import pytest

import paper_2111_06868_amd as sv
from paper_2111_06868_amd import _native as N
from oracle import brute, ref
from workloads import circuits as wc
from helpers import header_functions, to_binding


def test_library_exports_every_declared_symbol():
    L = N.lib()
    declared = header_functions()
    assert len(declared) >= 30
    for name in declared:
        assert hasattr(L, name), name
        assert name in N.SIGNATURES, name
    assert set(N.SIGNATURES) == set(declared)


def test_version():
    assert N.lib().sv_version() >= 1


@pytest.mark.parametrize("name,params", [
    ("I", ()), ("X", ()), ("Y", ()), ("Z", ()), ("H", ()), ("SQRT_X", ()), ("SQRT_Y", ()),
    ("SQRT_W", ()), ("RX", (0.37,)), ("RY", (-2.1,)), ("RZ", (5.5,)), ("CZ", ()), ("CX", ()),
    ("CPHASE", (1.3,)), ("SWAP", ()), ("FSIM", (math.pi / 2, math.pi / 6)), ("FSIM", (0.3, 2.9)),
])
def test_gate_table_matches_oracle(name, params):
    k = 1 if name in ("I", "X", "Y", "Z", "H", "SQRT_X", "SQRT_Y", "SQRT_W", "RX", "RY", "RZ") else 2
    got = sv.gate_matrix((name, tuple(range(k)), params))
    assert np.max(np.abs(got - ref.gate_matrix(name, params))) <= 1e-15


def test_matrix_gate_roundtrip():
    M = wc.haar_unitary_from_seed(5, 3)
    got = sv.gate_matrix(("MATRIX", (0, 1, 2), (), -1, M))
    assert np.array_equal(got, M)


def test_fuse_paper_compress_example():
    """Circuit utilities section: compress(max_n_qubits=3) prints blocks
    (0,1,2), (0,3,4), (1,3,4), (2,3,4)."""
    gates = to_binding(wc.paper_compress_example())
    plan = sv.fuse(gates, 5, 3, sv.RULE_PAPER)
    assert [b.qubits for b in plan.blocks(False)] == [(0, 1, 2), (0, 3, 4), (1, 3, 4), (2, 3, 4)]


@pytest.mark.parametrize("seed", range(4))
def test_fuse_paper_rule_matches_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    n = 9
    gates = wc.random_gate_list(n, 60, rng, max_k=2)
    for k in range(2, 7):
        plan = sv.fuse(to_binding(gates), n, k, sv.RULE_PAPER)
        want = ref.fuse_paper([g.qubits for g in gates], k)
        got = [(b.qubits, b.members) for b in plan.blocks(False)]
        assert got == [(q, m) for q, m in want]


def test_fused_block_matrices_match_oracle():
    rng = np.random.default_rng(7)
    n = 8
    gates = wc.random_gate_list(n, 40, rng, max_k=3)
    ops = [(ref.matrix_of(g), g.qubits) for g in gates]
    for k in (3, 4, 6):
        plan = sv.fuse(to_binding(gates), n, k, sv.RULE_PAPER)
        for b in plan.blocks():
            want = ref.block_matrix([ops[i] for i in b.members], b.qubits)
            assert np.max(np.abs(b.matrix - want)) <= 1e-13


@pytest.mark.parametrize("rule", [sv.RULE_PAPER, sv.RULE_ENHANCED, sv.RULE_NONE])
def test_plan_product_equals_circuit_unitary(rule):
    """Several plans are correct; each must reproduce the circuit's unitary."""
    rng = np.random.default_rng(11)
    for n in (5, 7):
        gates = wc.random_gate_list(n, 30, rng, max_k=2)
        U = brute.circuit_unitary(n, [(ref.matrix_of(g), g.qubits) for g in gates])
        for k in (2, 3, 5):
            plan = sv.fuse(to_binding(gates), n, k, rule)
            blocks = plan.blocks()
            assert sorted(i for b in blocks for i in b.members) == list(range(len(gates)))
            for b in blocks:
                assert rule == sv.RULE_NONE or len(b.qubits) <= k
                assert all(set(gates[i].qubits) <= set(b.qubits) for i in b.members)
            V = brute.circuit_unitary(n, [(b.matrix, b.qubits) for b in blocks])
            assert np.max(np.abs(V - U)) <= 1e-12


def test_enhanced_rule_never_needs_more_passes():
    for cfg in (0, 1, 2):
        n, gates = wc.config_circuit(cfg)
        g = to_binding(gates)
        for k in (2, 3, 4, 5, 6):
            p = len(sv.fuse(g, n, k, sv.RULE_PAPER))
            e = len(sv.fuse(g, n, k, sv.RULE_ENHANCED))
            assert e <= p, (cfg, k, e, p)
        assert len(sv.fuse(g, n, 2, sv.RULE_NONE)) == len(gates)


def test_paper_rule_pass_counts_on_workloads():
    for cfg in (1, 2):
        n, gates = wc.config_circuit(cfg)
        for k in (2, 3, 4, 5, 6):
            got = len(sv.fuse(to_binding(gates), n, k, sv.RULE_PAPER))
            assert got == len(ref.fuse_paper([x.qubits for x in gates], k))


# ------------------------------------------------------------ argument checks
def _gate(kind, qubits, params=(0.0, 0.0)):
    g = N.sv_gate()
    g.kind = N.GATE_KINDS[kind]
    g.k = len(qubits)
    for j, q in enumerate(qubits):
        g.q[j] = q
    g.params[0], g.params[1] = params
    g.param = -1
    return g


def _fuse_rc(gates, n, k=3, rule=N.RULE_PAPER):
    arr = (N.sv_gate * len(gates))(*gates)
    h = ctypes.c_void_p()
    rc = N.lib().sv_fuse(ctypes.cast(arr, ctypes.POINTER(N.sv_gate)), len(gates), n, k, rule, ctypes.byref(h))
    if rc == 0:
        N.lib().sv_plan_free(h)
    return rc


def test_validation_error_codes():
    assert _fuse_rc([_gate("H", (0,))], 4) == N.OK
    assert _fuse_rc([_gate("H", (4,))], 4) == N.ERR_QUBIT          # out of range
    assert _fuse_rc([_gate("CZ", (1, 1))], 4) == N.ERR_QUBIT       # repeated
    g = _gate("CZ", (0, 1)); g.k = 1
    assert _fuse_rc([g], 4) == N.ERR_ARG                           # arity mismatch
    g = _gate("H", (0,)); g.kind = 99
    assert _fuse_rc([g], 4) == N.ERR_ARG                           # unknown kind
    g = _gate("RX", (0,), (float("nan"), 0.0))
    assert _fuse_rc([g], 4) == N.ERR_ARG                           # non-finite parameter
    g = _gate("CZ", (0, 1)); g.param = 0
    assert _fuse_rc([g], 4) == N.ERR_ARG                           # param on a non-rotation
    g = _gate("H", (0,)); g.kind = 0; g.k = 1; g.m = None
    assert _fuse_rc([g], 4) == N.ERR_ARG                           # matrix gate without matrix
    assert _fuse_rc([_gate("CZ", (0, 1))], 4, k=1) == N.ERR_ARG    # gate larger than max_k
    assert _fuse_rc([_gate("H", (0,))], 4, k=7) == N.ERR_ARG
    assert _fuse_rc([_gate("H", (0,))], 4, rule=9) == N.ERR_ARG
    assert "max_k" in N.lib().sv_last_error().decode() or N.lib().sv_last_error()


def test_alloc_rejects_bad_arguments_before_device_work():
    L = N.lib()
    h = ctypes.c_void_p()
    assert L.sv_alloc(0, N.C64, None, 0, None, ctypes.byref(h)) == N.ERR_ARG
    assert L.sv_alloc(36, N.C64, None, 0, None, ctypes.byref(h)) == N.ERR_ARG
    assert L.sv_alloc(35, N.C128, None, 0, None, ctypes.byref(h)) == N.ERR_ARG
    assert L.sv_alloc(4, 7, None, 0, None, ctypes.byref(h)) == N.ERR_ARG
    # a buffer too small for the state (the pointer is never dereferenced)
    assert L.sv_alloc(10, N.C64, ctypes.c_void_p(4096), 8 * 1023, None, ctypes.byref(h)) == N.ERR_SIZE
    assert L.sv_alloc(10, N.C64, ctypes.c_void_p(4096 + 8), 1 << 20, None, ctypes.byref(h)) == N.ERR_ARG
    assert L.sv_alloc(4, N.C64, None, 0, None, None) == N.ERR_ARG
    assert h.value is None


def test_batch_description_validation():
    """sv_batch_required_bytes checks the description on the host: sizes
    (each state 256-byte aligned), precision, max_k, offsets and gates."""
    L = N.lib()
    ga = sv.GateArray([("H", (0,)), ("CZ", (0, 1)), ("H", (2,))])
    nq = np.array([2, 3], dtype=np.int32)
    offs = np.array([0, 2, 3], dtype=np.int64)

    def desc(**kw):
        d = N.sv_batch_desc()
        d.n_traj = 2
        d.max_k = kw.get("max_k", -1)
        d.n_qubits = kw.get("nq", nq).ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.gate_offsets = kw.get("offs", offs).ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.gates = ga.ptr
        d.precision = kw.get("precision", 0)
        return d

    need = ctypes.c_size_t()
    assert L.sv_batch_required_bytes(ctypes.byref(desc()), ctypes.byref(need)) == N.OK
    assert need.value == 256 + 256  # 4 and 8 complex64 amplitudes, each padded to 256 bytes
    for prec in (sv.PREC_SPLIT_BF16, sv.PREC_SPLIT_FP16):
        assert L.sv_batch_required_bytes(ctypes.byref(desc(precision=prec)), ctypes.byref(need)) == N.OK
    for prec in (sv.PREC_FP64, 7):
        assert L.sv_batch_required_bytes(ctypes.byref(desc(precision=prec)), ctypes.byref(need)) == N.ERR_ARG
    assert "precision" in L.sv_last_error().decode()
    assert L.sv_batch_required_bytes(ctypes.byref(desc(max_k=0)), ctypes.byref(need)) == N.ERR_ARG
    bad_offs = np.array([0, 1, 0], dtype=np.int64)  # trajectory 1 ends before it starts
    assert L.sv_batch_required_bytes(ctypes.byref(desc(offs=bad_offs)), ctypes.byref(need)) == N.ERR_ARG
    small = np.array([1, 3], dtype=np.int32)  # CZ on qubit 1 of a 1-qubit trajectory
    assert L.sv_batch_required_bytes(ctypes.byref(desc(nq=small)), ctypes.byref(need)) == N.ERR_QUBIT
    assert L.sv_batch_required_bytes(ctypes.byref(desc()), None) == N.ERR_ARG


def test_binding_raises_value_error_for_bad_input():
    with pytest.raises(ValueError):
        sv.fuse([("H", (9,))], 4, 2)
    with pytest.raises(ValueError):
        sv.gate_matrix(("NOPE", (0,)))


def test_positions_follow_paper_order():
    # Grover example: order [0, 1, 2] puts qubit 0 at the most significant bit
    assert sv.positions([0, 1, 2], [1, 2]) == (1, 0)
    assert sv.positions(["a", "b"], ["a"]) == (1,)


def test_auto_rule_picks_a_valid_plan():
    """SV_RULE_AUTO with max_k = -1 chooses a rule and k from the (default)
    cost table; the plan it returns must still equal the circuit."""
    rng = np.random.default_rng(21)
    n = 6
    gates = wc.random_gate_list(n, 40, rng, max_k=2)
    plan = sv.fuse(to_binding(gates), n, -1, sv.RULE_AUTO)
    assert plan.rule in (sv.RULE_ENHANCED, sv.RULE_TILED)
    assert 2 <= plan.max_k <= 6
    U = brute.circuit_unitary(n, [(ref.matrix_of(g), g.qubits) for g in gates])
    V = brute.circuit_unitary(n, [(b.matrix, b.qubits) for b in plan.blocks()])
    assert np.max(np.abs(V - U)) <= 1e-12
    # on the 30-qubit workload the tiled plan is priced cheaper by default
    n30, g30 = wc.config_circuit(1)
    p30 = sv.fuse(to_binding(g30), n30, -1, sv.RULE_AUTO)
    assert p30.rule == sv.RULE_TILED and p30.max_k <= 4


def test_tile_shape_validation():
    """Only the compiled tile shapes are accepted; the call launches nothing."""
    for shape in sv.TILE_SHAPES:
        sv.set_tile_shape(*shape)
    sv.set_tile_shape(14, 16)
    for bad in ((14, 4), (12, 8), (13, 2), (15, 8), (13, 16), (14, 32)):
        with pytest.raises(ValueError):
            sv.set_tile_shape(*bad)


def _valid_order(gates, order):
    """Every qubit's gates appear in circuit order (so the product is kept)."""
    last = {}
    for gi in order:
        for q in gates[gi].qubits:
            if last.get(q, -1) > gi:
                return False
            last[q] = gi
    return True


def _tile_runs(union, tile_bits=14):
    """log2 of the run length of the tile of a union: the union plus its
    lowest missing positions, tile_bits in all, then count 0, 1, .. in a row."""
    tile = set(union)
    p = 0
    while len(tile) < tile_bits:
        tile.add(p)
        p += 1
    r = 0
    while r in tile:
        r += 1
    return r


def _pass_fits(union, limit=10, tile_bits=14):
    # the default union limit 10: a tile of 128-byte runs (2^4 amplitudes) or longer
    return len(union) <= tile_bits and _tile_runs(union, tile_bits) >= tile_bits - limit


def test_tile_runs_of_small_unions():
    """Every union of at most 10 positions gives runs of at least 2^4 amplitudes,
    so the tile-fit rule only widens the old 10-position limit."""
    rng = np.random.default_rng(5)
    for _ in range(2000):
        u = set(rng.choice(30, size=int(rng.integers(1, 11)), replace=False).tolist())
        assert _pass_fits(u)
    assert _tile_runs(range(14)) == 14 and _tile_runs(range(16, 30)) == 0
    assert _pass_fits(set(range(4)) | set(range(20, 30))) and not _pass_fits(set(range(3)) | set(range(19, 30)))


@pytest.mark.parametrize("cfg", [1, 2])
def test_tiled_plan_structure(cfg):
    """SV_RULE_TILED: passes whose tiles are made of runs of at least 2^4
    amplitudes (the default union limit 10: every union of <= 10 positions,
    and larger ones holding enough low positions), made of blocks of <= 4
    qubits, consecutive, with every gate once and each qubit's gates in
    order."""
    n, gates = wc.config_circuit(cfg)
    plan = sv.fuse(to_binding(gates), n, 4, sv.RULE_TILED)
    blocks = plan.blocks(False)
    order = [i for b in blocks for i in b.members]
    assert sorted(order) == list(range(len(gates)))
    assert _valid_order(gates, order)
    passes = {}
    prev = None
    for b in blocks:
        assert len(b.qubits) <= 4
        if b.tile_pass >= 0:
            assert b.tile_pass not in passes or prev == b.tile_pass  # consecutive
            passes.setdefault(b.tile_pass, set()).update(b.qubits)
        prev = b.tile_pass
    assert passes and all(_pass_fits(u) for u in passes.values())
    assert any(len(u) > 10 for u in passes.values())  # the grid circuits use the wider unions
    # at most one launch's capacity of blocks per pass
    cap = sv.get_tile_shape()[2]
    per_pass = {}
    for b in blocks:
        if b.tile_pass >= 0:
            per_pass[b.tile_pass] = per_pass.get(b.tile_pass, 0) + 1
    assert max(per_pass.values()) <= cap
    # no block of fewer than 4 qubits could have joined the nearest earlier
    # block sharing a qubit with it
    for i, b in enumerate(blocks):
        m = set(b.qubits)
        prev_b = next((blocks[j] for j in range(i - 1, -1, -1) if set(blocks[j].qubits) & m), None)
        if prev_b is not None and len(m | set(prev_b.qubits)) <= 4:
            u = passes.get(prev_b.tile_pass, set(prev_b.qubits))
            assert prev_b.tile_pass >= 0 and not _pass_fits(u | m)
    n_launch = len(passes) + sum(1 for b in blocks if b.tile_pass < 0)
    # far fewer state passes than blocks (30 q: 22 passes for 845 gates)
    assert n_launch <= len(blocks) // 3


@pytest.mark.parametrize("rule", [sv.RULE_TILED, sv.RULE_ENHANCED])
def test_frontier_plans_equal_circuit_unitary(rule):
    rng = np.random.default_rng(31)
    for n in (6, 8):
        gates = wc.random_gate_list(n, 50, rng, max_k=2)
        U = brute.circuit_unitary(n, [(ref.matrix_of(g), g.qubits) for g in gates])
        for k in (2, 3, 4):
            blocks = sv.fuse(to_binding(gates), n, k, rule).blocks()
            assert _valid_order(gates, [i for b in blocks for i in b.members])
            V = brute.circuit_unitary(n, [(b.matrix, b.qubits) for b in blocks])
            assert np.max(np.abs(V - U)) <= 1e-12


def test_enhanced_rule_frontier_counts():
    """The enhanced rule keeps the cheaper of its two candidate plans; on the
    30-qubit workload the frontier plan wins for k >= 4."""
    n, gates = wc.config_circuit(1)
    got = [len(sv.fuse(to_binding(gates), n, k, sv.RULE_ENHANCED)) for k in (4, 5, 6)]
    paper = [len(sv.fuse(to_binding(gates), n, k, sv.RULE_PAPER)) for k in (4, 5, 6)]
    assert all(g < p for g, p in zip(got, paper)), (got, paper)


def test_plans_per_precision():
    """sv_fuse_prec: the tiled rule fills passes up to one launch of the
    precision's operands (split BF16: 5 blocks; FP32 and split FP16, whose
    operands are smaller: 7), with every gate once in circuit order."""
    n, gates = wc.config_circuit(1)
    g = to_binding(gates)
    counts = {}
    for prec, cap in ((sv.PREC_SPLIT_BF16, 5), (sv.PREC_SPLIT_BF16X3, 5), (sv.PREC_FP32, 7),
                      (sv.PREC_SPLIT_FP16, 7), (None, 5)):
        blocks = sv.fuse(g, n, 4, sv.RULE_TILED, precision=prec).blocks(False)
        order = [i for b in blocks for i in b.members]
        assert sorted(order) == list(range(len(gates))) and _valid_order(gates, order)
        per_pass, unions = {}, {}
        for b in blocks:
            if b.tile_pass >= 0:
                per_pass[b.tile_pass] = per_pass.get(b.tile_pass, 0) + 1
                unions.setdefault(b.tile_pass, set()).update(b.qubits)
        assert max(per_pass.values()) <= cap and all(_pass_fits(u) for u in unions.values())
        counts[prec] = (len(per_pass), max(per_pass.values()))
    assert counts[sv.PREC_SPLIT_FP16][1] > 5 and counts[sv.PREC_SPLIT_FP16][0] < counts[None][0]
    for bad in (9, -1):
        with pytest.raises(ValueError):
            sv.fuse(g, n, 4, sv.RULE_TILED, precision=bad)


def test_small_states_keep_the_union_limit():
    """Below 14 qubits no tile holds a pass, and the tiled rule keeps to unions
    of at most the limit (10); at 14 qubits and above wider unions appear."""
    rng = np.random.default_rng(77)
    for n, wide in ((12, False), (13, False), (16, True)):
        gates = wc.random_gate_list(n, 30 * n, rng, max_k=2)
        blocks = sv.fuse(to_binding(gates), n, 4, sv.RULE_TILED, precision=sv.PREC_SPLIT_FP16).blocks(False)
        unions = {}
        for b in blocks:
            if b.tile_pass >= 0:
                unions.setdefault(b.tile_pass, set()).update(b.qubits)
        assert unions and all(_pass_fits(u) for u in unions.values())
        assert (max(len(u) for u in unions.values()) > 10) == wide, (n, sorted(len(u) for u in unions.values()))


def test_tile_union_setting():
    """The tiled rule keeps every pass's tile to runs of at least
    2^(14 - limit) amplitudes for the configured union limit."""
    n, gates = wc.config_circuit(2)
    g = to_binding(gates)
    counts = {}
    try:
        for u in (8, 9, 10):
            sv.set_tile_union(u)
            blocks = sv.fuse(g, n, 4, sv.RULE_TILED).blocks(False)
            unions = {}
            for b in blocks:
                if b.tile_pass >= 0:
                    unions.setdefault(b.tile_pass, set()).update(b.qubits)
            assert all(_pass_fits(x, limit=u) for x in unions.values())
            counts[u] = len(unions) + sum(1 for b in blocks if b.tile_pass < 0)
        for bad in (7, 11, 0):
            with pytest.raises(ValueError):
                sv.set_tile_union(bad)
    finally:
        sv.set_tile_union(10)
    assert counts[8] >= counts[9] >= counts[10]
