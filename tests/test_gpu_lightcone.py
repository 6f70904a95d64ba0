"""The 512 noisy trajectories cut to the light cone of qubit 0 (the paper's
pop, sv_lightcone) and moved onto the cone's qubits (sv_compact_qubits), run
by the batch kernels on the GPU, against the oracle's <Z_0> of every FULL
trajectory (stored by tests/golden/make_full_size_golden.py)."""
import os

import numpy as np
import pytest

import paper_2111_06868_amd as sv
from workloads import circuits as wc

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trajectories512_z0.txt")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield
    torch.cuda.synchronize()


def _golden():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    mean = float(rows[0][1])
    z = np.array([float(r[2]) for r in rows[1:]])
    n = [int(r[1]) for r in rows[1:]]
    return mean, n, z


@pytest.mark.parametrize("precision", [sv.PREC_FP32, sv.PREC_SPLIT_BF16])
def test_lightcone_trajectories_vs_oracle_full_circuits(precision):
    mean, n_ref, z_ref = _golden()
    trajs = wc.trajectory_batch()
    assert [t.n for t in trajs] == n_ref
    cut = []
    for t in trajs:
        gates = [(g.name, g.qubits, g.params) for g in t.gates]
        keep = sv.lightcone(gates, t.n, (0,))
        n_used, moved, pos = sv.compact_qubits([gates[i] for i in keep], t.n, (0,))
        assert pos[0] == 0
        cut.append((n_used, moved))
    assert sum(1 << n for n, _ in cut) < sum(1 << t.n for t in trajs)
    z = sv.Batch(cut, max_k=-1, precision=precision).run(use_graph=True)
    err = float(np.abs(z - z_ref).max())
    print("[parity] light-cone trajectories (precision %d) vs oracle full circuits: max |dZ0| %.3e, "
          "mean %.6f (oracle %.6f), amplitudes %d -> %d" % (precision, err, z.mean(), mean,
                                                           sum(1 << t.n for t in trajs),
                                                           sum(1 << n for n, _ in cut)), flush=True)
    assert err <= 1e-5
    assert abs(z.mean() - mean) <= 1e-6
