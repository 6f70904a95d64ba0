"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
catch each one: every mutant must make at least one pin fail."""
import math

import numpy as np
import pytest

import oracle_pins as P
from oracle import ref

_orig_apply = ref.apply
_orig_run = ref.run_matrices
_orig_gate = ref.gate_matrix
_orig_product = ref.product_state
_orig_expect = ref.expectation
_orig_fuse = ref.fuse_paper


def _map_ops(fn):
    def run(psi, ops):
        n = int(psi.size).bit_length() - 1
        return _orig_run(psi, [fn(n, M, q) for M, q in ops])

    def apply(psi, M, q):
        n = int(psi.size).bit_length() - 1
        M2, q2 = fn(n, M, q)
        return _orig_apply(psi, M2, q2)
    return run, apply


def mut_local_bit_order(mp):
    """q[0] taken as the least significant local bit."""
    run, apply = _map_ops(lambda n, M, q: (M, tuple(reversed(q))))
    mp.setattr(ref, "run_matrices", run)
    mp.setattr(ref, "apply", apply)


def mut_transposed_matrix(mp):
    run, apply = _map_ops(lambda n, M, q: (np.asarray(M).T.copy(), q))
    mp.setattr(ref, "run_matrices", run)
    mp.setattr(ref, "apply", apply)


def mut_position_mirror(mp):
    """Index bit n-1-p used for position p (global bit order flipped)."""
    run, apply = _map_ops(lambda n, M, q: (M, tuple(n - 1 - x for x in q)))
    mp.setattr(ref, "run_matrices", run)
    mp.setattr(ref, "apply", apply)


def mut_conjugated_gates(mp):
    mp.setattr(ref, "gate_matrix", lambda name, params=(): _orig_gate(name, params).conj())


def mut_fsim_sign(mp):
    def g(name, params=()):
        M = _orig_gate(name, params)
        if name.upper() == "FSIM":
            M = M.copy()
            M[1, 2] = -M[1, 2]
            M[2, 1] = -M[2, 1]
        return M
    mp.setattr(ref, "gate_matrix", g)


def mut_rotation_full_angle(mp):
    def g(name, params=()):
        if name.upper() in ("RX", "RY", "RZ"):
            return _orig_gate(name, (2 * float(params[0]),))
        return _orig_gate(name, params)
    mp.setattr(ref, "gate_matrix", g)


def mut_sqrt_w_unnormalised(mp):
    def g(name, params=()):
        if name.upper() == "SQRT_W":
            W = ref.PAULI["X"] + ref.PAULI["Y"]
            return ((1 + 1j) * np.eye(2) + (1 - 1j) * W) / 2
        return _orig_gate(name, params)
    mp.setattr(ref, "gate_matrix", g)


def mut_cx_control_swapped(mp):
    def g(name, params=()):
        if name.upper() == "CX":
            return np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=complex)
        return _orig_gate(name, params)
    mp.setattr(ref, "gate_matrix", g)


def mut_product_token_order(mp):
    mp.setattr(ref, "product_state",
               lambda n, tokens: _orig_product(n, tokens[::-1] if len(tokens) > 1 else tokens))


def mut_expectation_dropped_term(mp):
    mp.setattr(ref, "expectation", lambda psi, terms: _orig_expect(psi, list(terms)[:-1])
               if len(terms) > 1 else _orig_expect(psi, terms))


def mut_expectation_imag(mp):
    def e(psi, terms):
        return sum(c * ref.inner(psi, ref.pauli_apply(psi, f)).imag for c, f in terms) + \
            sum(c * ref.inner(psi, ref.pauli_apply(psi, f)).real for c, f in terms if len(f) == 0)
    mp.setattr(ref, "expectation", e)


def mut_fusion_append_current(mp):
    """The naive rule: keep appending to the current block until it overflows."""
    def fuse(qubit_lists, max_k):
        blocks = []
        for gi, qs in enumerate(qubit_lists):
            if blocks and len(blocks[-1][0] | set(qs)) <= max_k:
                blocks[-1][0].update(qs)
                blocks[-1][1].append(gi)
            else:
                blocks.append((set(qs), [gi]))
        return [(tuple(sorted(b)), m) for b, m in blocks]
    mp.setattr(ref, "fuse_paper", fuse)


def mut_fusion_first_intersecting(mp):
    """Merge into the FIRST intersecting block (illegal reordering)."""
    def fuse(qubit_lists, max_k):
        blocks = []
        for gi, qs in enumerate(qubit_lists):
            qs = set(qs)
            tgt = next((b for b in blocks if b["q"] & qs), None)
            if tgt is not None and len(tgt["q"] | qs) <= max_k:
                tgt["q"] |= qs
                tgt["m"].append(gi)
            else:
                blocks.append({"q": set(qs), "m": [gi]})
        return [(tuple(sorted(b["q"])), b["m"]) for b in blocks]
    mp.setattr(ref, "fuse_paper", fuse)


def mut_param_shift_wrong_shift(mp):
    def ps(n, gates, thetas, terms, indices=None, initial="0"):
        thetas = np.asarray(thetas, dtype=np.float64)
        idx = range(len(thetas)) if indices is None else indices
        out = []
        for p in idx:
            tp = thetas.copy(); tp[p] += math.pi / 4
            tm = thetas.copy(); tm[p] -= math.pi / 4
            out.append(0.5 * (ref.energy(n, gates, tp, terms, initial) - ref.energy(n, gates, tm, terms, initial)))
        return np.array(out)
    mp.setattr(ref, "param_shift_grad", ps)



def mut_fidelity_unsquared_overlap(mp):
    """|<ref|psi>| used where its square belongs (halves every small 1-F)."""
    def fe(r, psi):
        ov = ref.inner(r, psi.astype(np.complex128))
        return 1.0 - abs(ov) / math.sqrt(ref.norm2(r) * ref.norm2(psi.astype(np.complex128)))
    mp.setattr(ref, "fidelity_error", fe)


def mut_fidelity_unnormalised(mp):
    """The norms of the two states left out of 1-F."""
    def fe(r, psi):
        return 1.0 - abs(ref.inner(r, psi.astype(np.complex128))) ** 2
    mp.setattr(ref, "fidelity_error", fe)


def mut_fidelity_raw_renormalised(mp):
    """The raw error divided by ||psi||^2 as well (hides norm drift)."""
    def fe(r, psi):
        ov = ref.inner(r, psi.astype(np.complex128))
        return abs(1.0 - abs(ov) ** 2 / (ref.norm2(r) * ref.norm2(psi.astype(np.complex128))))
    mp.setattr(ref, "fidelity_error_raw", fe)


def mut_max_abs_real_part(mp):
    """Only real parts compared."""
    mp.setattr(ref, "max_abs", lambda r, psi: float(np.max(np.abs((r - psi.astype(np.complex128)).real))))

MUTANTS = [
    mut_local_bit_order, mut_transposed_matrix, mut_position_mirror,
    mut_conjugated_gates, mut_fsim_sign, mut_rotation_full_angle,
    mut_sqrt_w_unnormalised, mut_cx_control_swapped, mut_product_token_order,
    mut_expectation_dropped_term, mut_expectation_imag,
    mut_fusion_append_current, mut_fusion_first_intersecting,
    mut_param_shift_wrong_shift,
    mut_fidelity_unsquared_overlap, mut_fidelity_unnormalised,
    mut_fidelity_raw_renormalised, mut_max_abs_real_part,
]


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda f: f.__name__)
def test_mutant_is_caught(mutant, monkeypatch):
    mutant(monkeypatch)
    caught = []
    for check in P.ALL_CHECKS:
        try:
            check()
        except (AssertionError, ValueError, np.linalg.LinAlgError) as e:  # noqa: F841
            caught.append(check.__name__)
            break
    assert caught, "planted mistake %s passed every pin" % mutant.__name__
