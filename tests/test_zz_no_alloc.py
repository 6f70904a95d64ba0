"""The entry point that allocates nothing (sv_expectation_noalloc) against
sv_expectation on the same states: two calls in a row, the second on a smaller
state with fewer terms, the largest term count, and the host-side refusals."""
import ctypes

import numpy as np
import pytest

import paper_2111_06868_amd as sv
from paper_2111_06868_amd import _native as N
from oracle import ref
from workloads import circuits as wc
from helpers import to_binding

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield
    torch.cuda.synchronize()


def _random_terms(n, count, seed):
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(count):
        qs = rng.choice(n, size=int(rng.integers(1, min(n, 5) + 1)), replace=False)
        terms.append((float(rng.standard_normal()), tuple((int(q), "XYZ"[int(rng.integers(3))]) for q in qs)))
    return terms


def _prepared(n, dtype, seed):
    gates = wc.random_gate_list(n, 4 * n, np.random.default_rng(seed), max_k=2)
    st = sv.State(n, dtype).run(to_binding(gates), max_k=4, rule=sv.RULE_ENHANCED)
    return st


def test_noalloc_matches_expectation_twice_then_smaller():
    print("noalloc: 20-qubit c64 state, 300 terms; then 12-qubit c128 state, 7 terms", flush=True)
    st1 = _prepared(20, "c64", 11)
    H1 = sv.pauli_sum(_random_terms(20, 300, 12))
    want1 = st1.expectation(H1)
    got1 = sv.expectation_noalloc(st1.tensor, 20, H1)
    assert got1 == want1  # same kernels, same fixed-order reduction
    st2 = _prepared(12, "c128", 13)
    terms2 = _random_terms(12, 7, 14)
    H2 = sv.pauli_sum(terms2)
    want2 = st2.expectation(H2)
    got2 = sv.expectation_noalloc(st2.tensor, 12, H2)
    assert got2 == want2
    assert abs(got2 - ref.expectation(st2.read(), terms2)) <= 1e-12
    # the first state again: the scratch keeps no stale tables
    assert sv.expectation_noalloc(st1.tensor, 20, H1) == want1


def test_noalloc_largest_term_count():
    print("noalloc: 4096 terms on a 16-qubit c64 state", flush=True)
    st = _prepared(16, "c64", 21)
    H = sv.pauli_sum(_random_terms(16, 4096, 22))
    assert sv.expectation_noalloc(st.tensor, 16, H) == st.expectation(H)


def test_noalloc_refusals():
    st = _prepared(10, "c64", 31)
    H = sv.pauli_sum([(1.0, ((0, "Z"),))])
    L = N.lib()
    out = ctypes.c_double()
    p = st.tensor.data_ptr()
    assert L.sv_expectation_noalloc(ctypes.c_void_p(p + 8), 10, N.C64, None, H.ptr, ctypes.byref(out)) == N.ERR_ARG
    assert L.sv_expectation_noalloc(ctypes.c_void_p(p), 0, N.C64, None, H.ptr, ctypes.byref(out)) == N.ERR_ARG
    assert L.sv_expectation_noalloc(ctypes.c_void_p(p), 10, 7, None, H.ptr, ctypes.byref(out)) == N.ERR_ARG
    Hbad = sv.pauli_sum([(1.0, ((10, "X"),))])
    assert L.sv_expectation_noalloc(ctypes.c_void_p(p), 10, N.C64, None, Hbad.ptr, ctypes.byref(out)) == N.ERR_QUBIT
    big = sv.pauli_sum([(1.0, ((0, "Z"),))] * 4097)
    assert L.sv_expectation_noalloc(ctypes.c_void_p(p), 10, N.C64, None, big.ptr, ctypes.byref(out)) == N.ERR_ARG
    assert sv.expectation_noalloc(st.tensor, 10, H) == st.expectation(H)
