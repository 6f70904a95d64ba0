"""GPU: batched noisy trajectories and the autotuner, against the oracle."""
import os

import numpy as np
import pytest

import paper_2111_06868_amd as sv
from oracle import ref
from workloads import circuits as wc
from helpers import to_binding

pytestmark = pytest.mark.gpu


def _batch_inputs(trajs):
    return [(t.n, to_binding(t.gates)) for t in trajs]


@pytest.mark.parametrize("max_k", [1, 2, 3, 5, -1])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_small_vs_oracle(max_k, use_graph):
    trajs = wc.trajectory_batch(count=14, root_seed=77, p=0.2, n_range=(3, 17), depth_range=(2, 7))
    assert sum(t.n_inserted for t in trajs) > 0
    b = sv.Batch(_batch_inputs(trajs), max_k=max_k)
    for rep in range(2):
        z = b.run(use_graph=use_graph)
        for i, t in enumerate(trajs):
            want = ref.simulate(t.n, t.gates, "0")
            got = b.read(i)
            fe = ref.fidelity_error(want, got)
            assert fe <= 1e-5, (i, t.n, fe)
            assert abs(z[i] - ref.z0(want)) <= 1e-5, (i, z[i], ref.z0(want))
    print("[parity] batch max_k=%s graph=%s ok" % (max_k, use_graph), flush=True)


@pytest.mark.parametrize("max_k", [3, -1])
@pytest.mark.parametrize("precision", [sv.PREC_SPLIT_BF16, sv.PREC_SPLIT_FP16])
def test_batch_split_vs_oracle(max_k, precision):
    """Split-BF16 / FP16 tile passes for the large trajectories (n >= 14):
    every state against the oracle, at the split's tolerance."""
    trajs = wc.trajectory_batch(count=10, root_seed=91, p=0.2, n_range=(12, 18), depth_range=(3, 9))
    assert sum(1 for t in trajs if t.n >= 14) >= 5
    b = sv.Batch(_batch_inputs(trajs), max_k=max_k, precision=precision)
    z = b.run(use_graph=True)
    for i, t in enumerate(trajs):
        want = ref.simulate(t.n, t.gates, "0")
        got = b.read(i)
        fe = ref.fidelity_error(want, got)
        ma = float(np.max(np.abs(got - want)))
        assert fe <= 1e-6 and ma <= 1e-5, (i, t.n, fe, ma)
        assert abs(z[i] - ref.z0(want)) <= 1e-5, (i, z[i], ref.z0(want))
    print("[parity] batch split precision=%d max_k=%s ok" % (precision, max_k), flush=True)


def _golden_z0():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trajectories512_z0.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return float(rows[0][1]), [int(r[1]) for r in rows[1:]], np.array([float(r[2]) for r in rows[1:]])


@pytest.mark.parametrize("precision", [sv.PREC_FP32, sv.PREC_SPLIT_BF16, sv.PREC_SPLIT_FP16, sv.PREC_SPLIT_BF16X3])
def test_batch_full_size_vs_oracle(precision):
    """The 512-trajectory noisy batch (n in 10..22, depth 8..24, p = 1e-3):
    <Z_0> of every trajectory against the oracle's (stored by
    tests/golden/make_full_size_golden.py) to 1e-5, and the batch mean."""
    mean, n_ref, z_ref = _golden_z0()
    trajs = wc.trajectory_batch()
    assert [t.n for t in trajs] == n_ref
    b = sv.Batch(_batch_inputs(trajs), max_k=-1, precision=precision)
    z = b.run(use_graph=True)
    z2 = b.run(use_graph=True)
    assert np.array_equal(z, z2)
    err = np.abs(z - z_ref)
    print("[parity] batch 512 precision=%d: max |dZ0| = %.3e (n >= 14: %.3e), mean Z0 = %.8f (oracle %.8f)"
          % (precision, err.max(), max(err[i] for i, t in enumerate(trajs) if t.n >= 14), z.mean(), mean),
          flush=True)
    assert err.max() <= 1e-5
    assert abs(z.mean() - mean) <= 1e-6
    assert np.all(np.abs(z) <= 1 + 1e-6)
    # the stored values against the oracle itself on a few trajectories
    for i in (0, 7, 300):
        assert abs(ref.trajectory_z0(trajs[i]) - z_ref[i]) <= 1e-12


@pytest.mark.parametrize("precision", [sv.PREC_FP32, sv.PREC_SPLIT_BF16, sv.PREC_FP64, sv.PREC_SPLIT_BF16X3])
def test_autotune_then_fuse_auto(precision):
    n = 16
    dtype = "c128" if precision == sv.PREC_FP64 else "c64"
    scratch = sv.State(n, dtype)
    cost = sv.autotune(scratch, precision)
    print("[tune] n=%d precision=%d cost_ms=%s" % (n, precision, np.array2string(cost, precision=4)), flush=True)
    assert np.all(cost[1:] > 0)
    rng = np.random.default_rng(3)
    gates = wc.random_gate_list(n, 200, rng, max_k=2)
    want = ref.simulate(n, gates, "+")
    st = sv.State(n, dtype).set_product("+").run(to_binding(gates), max_k=-1, rule=sv.RULE_ENHANCED,
                                                 precision=precision)
    fe = ref.fidelity_error(want, st.read())
    assert fe <= (1e-12 if dtype == "c128" else 1e-5)


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    """sv_autotune records its table in $SV_TUNE_CACHE keyed by (architecture,
    n, precision); sv_tune_cache_load installs the records of this GPU's
    architecture only, and a later fusion with max_k = -1 uses them."""
    path = tmp_path / "tune.txt"
    path.write_text("sv-tune-1 gfx000 16 0" + " 1" * 22 + " 0" * 28 + " 0 256 14 16\n")
    monkeypatch.setenv("SV_TUNE_CACHE", str(path))
    n = 16
    cost = sv.autotune(sv.State(n, "c64"), sv.PREC_FP32)
    lines = [ln.split() for ln in path.read_text().splitlines()]
    mine = [ln for ln in lines if ln[1] != "gfx000"]
    assert len(lines) == 2 and len(mine) == 1
    assert mine[0][1].startswith("gfx9") and mine[0][2:4] == [str(n), str(sv.PREC_FP32)]
    assert np.allclose([float(x) for x in mine[0][4:10]], cost[1:], rtol=1e-15)
    # a second tuning replaces the record of its key
    sv.autotune(sv.State(n, "c64"), sv.PREC_FP32)
    assert len(path.read_text().splitlines()) == 2
    sv.set_cost_table(n, sv.PREC_FP32, np.array([0, 9, 9, 9, 9, 9, 9.0]))
    assert sv.tune_cache_load(str(path)) == 1
    rng = np.random.default_rng(4)
    gates = wc.random_gate_list(n, 120, rng, max_k=2)
    st = sv.State(n, "c64").run(to_binding(gates), max_k=-1, rule=sv.RULE_ENHANCED)
    assert ref.fidelity_error(ref.simulate(n, gates, "0"), st.read()) <= 1e-5
    with pytest.raises(sv.SvValueError):
        sv.tune_cache_load(str(tmp_path / "missing.txt"))


def test_native_library_is_loaded():
    import os
    from paper_2111_06868_amd import _native
    L = _native.lib()
    maps = open("/proc/self/maps").read()
    assert os.path.realpath(_native.LIB_PATH) in maps
    assert L.sv_version() >= 1


def test_batch_edge_trajectories():
    """Boundary sizes of the two batch paths (13: LDS-resident; 14: one tile;
    22: 256 tiles), trajectories without gates or with one gate."""
    rng = np.random.default_rng(91)
    G = wc.Gate
    trajs = [
        (13, []),
        (14, []),
        (14, [G("X", (0,))]),
        (15, [G("FSIM", (3, 14), (0.7, 0.3))]),
        (22, wc.random_gate_list(22, 40, rng, max_k=2)),
        (14, wc.random_gate_list(14, 60, rng, max_k=2)),
    ]
    b = sv.Batch([(n, to_binding(g)) for n, g in trajs], max_k=3)
    z = b.run(use_graph=True)
    for i, (n, gates) in enumerate(trajs):
        want = ref.simulate(n, gates, "0")
        got = b.read(i)
        fe = ref.fidelity_error(want, got)
        assert fe <= 1e-5, (i, n, fe)
        assert np.max(np.abs(got - want)) <= 1e-5, (i, n)
        assert abs(z[i] - ref.z0(want)) <= 1e-5, (i, z[i], ref.z0(want))
    assert abs(z[1] - 1.0) <= 1e-12 and abs(z[2] + 1.0) <= 1e-12
    print("[parity] batch edge trajectories ok", flush=True)
