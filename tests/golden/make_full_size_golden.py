"""Write the stored oracle values that the full-size GPU tests compare with.

Only the oracle (oracle/) and the seeded input generators (workloads/) are
called; nothing here touches the GPU library.  Run from the repository root:

    python tests/golden/make_full_size_golden.py [ansatz] [trajectories]

* ansatz20_gradients.txt: the 20-qubit hardware-efficient ansatz (12 layers of
  RY and RZ on every qubit plus a CZ ladder, 480 angles from seed 3) with
  H = sum_i Z_i Z_{i+1} + 0.5 sum_i X_i: the energy, and for every angle the
  parameter-shift derivative (exact for rotations exp(-i theta P / 2)) and the
  central finite difference with h = 1e-3.
* trajectories512_z0.txt: <Z_0> of each of the 512 noisy trajectories (n in
  10..22, depth 8..24, two-qubit depolarizing p = 1e-3 sampled per trajectory
  from SeedSequence(4)) evolved by the oracle one gate at a time, and their
  mean.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

H_STEP = 1e-3


def _ansatz_worker(p):
    from oracle import ref
    from workloads import circuits as wc
    gates, thetas = wc.ansatz_circuit(20, 12, seed=3)
    H = wc.ansatz_observable(20)
    ps = ref.param_shift_grad(20, gates, thetas, H, indices=[p])[0]
    fd = ref.fd_grad(20, gates, thetas, H, h=H_STEP, indices=[p])[0]
    return p, ps, fd


def _traj_worker(t):
    from oracle import ref
    from workloads import circuits as wc
    traj = wc.trajectory_batch()[t]
    return t, traj.n, ref.trajectory_z0(traj)


def write_ansatz(procs):
    from oracle import ref
    from workloads import circuits as wc
    gates, thetas = wc.ansatz_circuit(20, 12, seed=3)
    H = wc.ansatz_observable(20)
    e = ref.energy(20, gates, thetas, H)
    with mp.Pool(procs) as pool:
        rows = sorted(pool.map(_ansatz_worker, range(len(thetas)), chunksize=4))
    path = os.path.join(HERE, "ansatz20_gradients.txt")
    with open(path, "w") as f:
        f.write("# 20-qubit ansatz (12 layers: RY then RZ on qubits 0..19, CZ(i, i+1) ladder),\n")
        f.write("# 480 angles U[0, 2pi) from default_rng(3); H = sum_{i<19} Z_i Z_{i+1} + 0.5 sum_i X_i.\n")
        f.write("# Complex128 oracle, one gate at a time.  Columns: parameter index, parameter-shift\n")
        f.write("# derivative [E(t + pi/2) - E(t - pi/2)] / 2, central difference (h = %g).\n" % H_STEP)
        f.write("energy %.17g\n" % e)
        for p, ps, fd in rows:
            f.write("%d %.17g %.17g\n" % (p, ps, fd))
    print("wrote", path)


def write_trajectories(procs):
    import numpy as np
    from workloads import circuits as wc
    count = len(wc.trajectory_batch())
    with mp.Pool(procs) as pool:
        rows = sorted(pool.map(_traj_worker, range(count), chunksize=2))
    path = os.path.join(HERE, "trajectories512_z0.txt")
    with open(path, "w") as f:
        f.write("# 512 noisy ladder random circuits (n ~ U{10..22}, depth ~ U{8..24}, fSim(pi/2, pi/6)\n")
        f.write("# with a two-qubit depolarizing draw p = 1e-3 after each, SeedSequence(4).spawn(512)).\n")
        f.write("# Complex128 oracle, one gate at a time, from |0..0>.  Columns: trajectory, qubits, <Z_0>.\n")
        f.write("mean %.17g\n" % float(np.mean([z for _, _, z in rows])))
        for t, n, z in rows:
            f.write("%d %d %.17g\n" % (t, n, z))
    print("wrote", path)


if __name__ == "__main__":
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    what = sys.argv[1:] or ["ansatz", "trajectories"]
    procs = int(os.environ.get("GOLDEN_PROCS", os.cpu_count() or 1))
    if "trajectories" in what:
        write_trajectories(procs)
    if "ansatz" in what:
        write_ansatz(procs)
