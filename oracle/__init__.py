"""CPU oracle for state-vector simulation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library under
``paper_2111_06868_amd`` and never imports it.  Everything is complex128.

Modules:
  ref    -- plain gate-at-a-time evolution (C core in sv_ref.c), gate table,
            metrics, Pauli expectations, parameter-shift / finite-difference
            gradients, the paper's greedy fusion rule, trajectories.
  brute  -- the full 2^n x 2^n unitary built from Kronecker products (n <= 8).
  density -- density matrices: gates, Kraus / matrix super operators, the
            noise channels, Tr(rho H), and channels sampled on pure states.
  ops    -- projections, measurements and controlled gates.
"""
