"""Host checks of the tile passes' LDS placement (sv_tile_placement): the
placement is a permutation of the tile that keeps 16-byte pairs whole, the
tile bits are the blocks' union plus the lowest other positions, and, by an
independent model of the block loop's LDS addresses (the lane -> column and
row assignment of the split tile kernels, 16-byte accesses served 8 lanes
over 32 banks or 16 lanes over 64 banks), the chosen placement leaves no
bank conflicts on the passes of the benchmark circuits.  No device work."""
import numpy as np
import pytest

import paper_2111_06868_amd as sv
from paper_2111_06868_amd import _native as N
from workloads import circuits as wc


def _deposit(v, mask):
    r, m = 0, mask
    while m:
        low = m & -m
        if v & 1:
            r |= low
        v >>= 1
        m &= m - 1
    return r


def _apply(img, i):
    r, b = 0, 0
    while i:
        if i & 1:
            r ^= int(img[b])
        i >>= 1
        b += 1
    return r


def _lds_cycles(img, tbit, tb, waves):
    """Cycles over ideal of the block loop's 16-byte LDS reads and writes of
    one block (rows on tile bits tbit, ascending) in a split tile pass with
    2^tb amplitudes and `waves` waves, for both bank models."""
    nbw = (1 << (tb - 9)) // waves
    m = sum(1 << t for t in tbit)
    cmask = ((1 << tb) - 1) & ~m
    ncb = (1 << (tb - 4)) // 32
    cq = [_apply(img, _deposit((r // nbw) * 32 * nbw + r % nbw, cmask)) for r in range(ncb)]
    cl = [_apply(img, _deposit(l * nbw, cmask)) for l in range(32)]
    rb = [int(img[t]) for t in tbit]

    def row(j):
        r = 0
        for b in range(4):
            if (j >> b) & 1:
                r ^= rb[b]
        return r

    ins = []
    for w in (0, waves - 1):
        def lane_cols(q, extra):
            return np.array([(cl[l & 31] ^ cq[w * nbw + q] ^ (extra if l >> 5 else 0)) for l in range(64)])
        qs = range(nbw) if tbit[0] == 0 else range(0, nbw, 2)
        rows_r = [8 * i + 2 * k for i in range(2) for k in range(2)] if tbit[0] == 0 else \
            [8 * i + t for i in range(2) for t in range(4)]
        rows_w = [4 * g for g in range(4)] if tbit[0] == 0 else [4 * g + e for g in range(4) for e in range(2)]
        for q in qs:
            lr, lw = lane_cols(q, rb[2]), lane_cols(q, rb[1])
            ins += [(row(j) ^ lr) * 8 for j in rows_r]
            ins += [(row(j) ^ lw) * 8 for j in rows_w]
    out = []
    for group, banks in ((8, 32), (16, 64)):
        act = 0
        for a in ins:
            for g0 in range(0, 64, group):
                dw = (a[g0:g0 + group, None] // 4 + np.arange(4)[None, :]).reshape(-1)
                per_bank = {}
                for d in set(dw.tolist()):
                    per_bank[d % banks] = per_bank.get(d % banks, 0) + 1
                act += max(per_bank.values())
        out.append(act / (len(ins) * 64 // group))
    return out


def _passes(cfg, precision=None):
    """Padded 4-position blocks of every tile pass of a benchmark circuit
    (planned for `precision`: the plan a run in it forms)."""
    n, gates = wc.config_circuit(cfg)
    plan = sv.fuse([(g.name, g.qubits, g.params) for g in gates], n, 4, sv.RULE_TILED, precision=precision)
    passes = {}
    for b in plan.blocks(False):
        passes.setdefault(b.tile_pass, []).append(b.qubits)
    out = []
    for p, blocks in sorted(passes.items()):
        um = 0
        for q in blocks:
            for x in q:
                um |= 1 << x
        pos = 0
        while bin(um).count("1") < 4:
            um |= 1 << pos
            pos += 1
        padded = []
        for q in blocks:
            pm = sum(1 << x for x in q)
            for x in range(n):
                if bin(pm).count("1") >= 4:
                    break
                if (um >> x) & 1 and not (pm >> x) & 1:
                    pm |= 1 << x
            padded.append([x for x in range(n) if (pm >> x) & 1])
        out.append((n, padded))
    return out


def test_placement_is_a_permutation_keeping_pairs():
    rng = np.random.default_rng(5)
    for trial in range(20):
        n = int(rng.integers(14, 33))
        union = sorted(rng.choice(n, size=int(rng.integers(4, 11)), replace=False).tolist())
        blocks = [sorted(rng.choice(union, size=4, replace=False).tolist()) for _ in range(int(rng.integers(1, 6)))]
        for tb, waves in ((14, 16), (14, 8), (13, 4), (13, 8)):
            tp, img, _ = sv.tile_placement(blocks, n, tb, waves)
            used = sorted(set(x for b in blocks for x in b))
            rest = [x for x in range(n) if x not in used][:tb - len(used)]
            assert tp.tolist() == sorted(used + rest)
            assert int(img[0]) == 1 and all(int(v) % 2 == 0 for v in img[1:])
            full = np.zeros(1 << tb, dtype=np.int64)
            for b in range(tb):
                full[((np.arange(1 << tb) >> b) & 1).astype(bool)] ^= int(img[b])
            assert np.array_equal(np.sort(full), np.arange(1 << tb))


@pytest.mark.parametrize("cfg,precision,most", [(1, None, 0), (2, None, 0), (1, sv.PREC_SPLIT_FP16, 2),
                                                (2, sv.PREC_SPLIT_FP16, 0)])
def test_benchmark_passes_bank_conflicts(cfg, precision, most):
    """The library's count of extra LDS cycles equals what the address model
    finds (per block: cycles over ideal - 1, summed over both bank models),
    and the benchmark circuits' passes have at most `most` in all (the split
    FP16 plans hold up to 7 blocks a pass, which leaves the search fewer
    conflict-free placements)."""
    total = 0
    tprec = sv.PREC_SPLIT_BF16 if precision is None else precision
    for n, blocks in _passes(cfg, precision):
        tp, img, conflicts = sv.tile_placement(blocks, n, 14, 16, tprec)
        model = 0.0
        for b in blocks:
            tbit = [tp.tolist().index(x) for x in b]
            model += sum(c - 1.0 for c in _lds_cycles(img, tbit, 14, 16))
        assert conflicts == model
        total += conflicts
    assert total <= most


def test_default_placement_had_conflicts_and_model_agrees():
    """The fixed placement (tile bits 5..8 XORed onto 1..4) leaves conflicts
    on a block with rows on tile bits (2, 3, 9, 12); the chosen one has none,
    and the library's count is zero exactly when the address model finds
    none."""
    blocks = [[2, 3, 9, 12]]
    tp, img, conflicts = sv.tile_placement(blocks, 20, 14, 16)
    assert conflicts == 0
    assert max(_lds_cycles(img, [2, 3, 9, 12], 14, 16)) == 1.0
    fixed = [(1 << b) ^ (((1 << b) >> 4) & 0x1E) for b in range(14)]
    assert max(_lds_cycles(fixed, [2, 3, 9, 12], 14, 16)) > 1.0


@pytest.mark.parametrize("tb,waves,cap", [(14, 8, 5), (13, 4, 2), (13, 8, 5)])
def test_other_shapes_free_of_bank_conflicts(tb, waves, cap):
    for n, blocks in _passes(1)[:8]:
        blocks = blocks[:cap]
        u = set(q for b in blocks for q in b)
        if len(u) > tb or (len(u) == tb and 0 not in u):
            continue  # no tb-bit tile holds it with position 0 as tile bit 0
        tp, img, conflicts = sv.tile_placement(blocks, n, tb, waves)
        assert conflicts == 0
        for b in blocks:
            tbit = [tp.tolist().index(x) for x in b]
            assert max(_lds_cycles(img, tbit, tb, waves)) == 1.0


def test_three_part_split_uses_the_split_placement():
    for n, blocks in _passes(1)[:6]:
        a = sv.tile_placement(blocks, n, 14, 16, sv.PREC_SPLIT_BF16)
        b = sv.tile_placement(blocks, n, 14, 16, sv.PREC_SPLIT_BF16X3)
        assert np.array_equal(a[1], b[1]) and a[2] == b[2] == 0


def test_fp32_keeps_the_fixed_placement_and_refusals():
    tp, img, c = sv.tile_placement([[0, 1, 2, 3]], 16, 14, 16, sv.PREC_FP32)
    assert c == 0 and [int(v) for v in img] == [(1 << b) ^ (((1 << b) >> 4) & 0x1E) for b in range(14)]
    with pytest.raises(N.SvError):
        sv.tile_placement([[0, 1, 2, 3]], 16, 12, 16)
    with pytest.raises(N.SvError):
        sv.tile_placement([[0, 1, 1, 2]], 16, 14, 16)
    with pytest.raises(N.SvError):
        sv.tile_placement([[0, 1, 2, 3]], 16, 14, 16, sv.PREC_FP64)
