"""Trajectories cut to the light cone of qubit 0 (the paper's pop) and moved
onto the cone's qubits give the same <Z_0> per trajectory as the full
trajectories, both run by the batch kernels on the GPU."""
import numpy as np
import pytest

import bench
import paper_2111_06868_amd as sv
from workloads import circuits as wc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield
    torch.cuda.synchronize()


def test_lightcone_trajectories_keep_z0():
    trajs = wc.trajectory_batch(count=48, root_seed=11)
    full = [(t.n, [(g.name, g.qubits, g.params) for g in t.gates]) for t in trajs]
    cut = [bench.lightcone_circuit(n, gs) for n, gs in full]
    assert sum(n for n, _ in cut) < sum(n for n, _ in full)
    z_full = sv.Batch(full, max_k=4).run()
    z_cut = sv.Batch(cut, max_k=4).run()
    err = float(np.abs(z_full - z_cut).max())
    print("[parity] light-cone trajectories: max |dZ0| %.3e, qubits %d -> %d"
          % (err, sum(n for n, _ in full), sum(n for n, _ in cut)), flush=True)
    assert err <= 1e-5
