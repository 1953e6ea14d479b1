"""Pins of the reference solver's grid structure (Sec. 2.5 and 2.6 of the paper).

- the added coarse grids reproduce table coarse-grid-example exactly;
- the padded block storage reproduces the one-ghost column of table ghost-cell-cost;
- refined trees are 2:1 balanced across faces, edges and corners, tile the domain, and
  equal a brute-force closure of the refinement predicate on tiny inputs.
"""
import itertools

import numpy as np
import pytest

from conftest import read_golden
from oracle import DIRICHLET, PERIODIC, OracleTree


def test_coarse_grid_table():
    rows = read_golden("coarse_grid_table.txt")
    t = OracleTree(2, (192, 96), (0, 0), (2, 1), [DIRICHLET] * 4, bs=8)
    base = t.base_level
    assert t.num_levels == len(rows)
    for paper_level, nx, ny, bs, nbx, nby in rows:
        l = base + (paper_level - 1)
        got_bs, ncell, nblocks = t.level_info(l)
        assert got_bs == bs
        assert ncell[:2] == (nx, ny)
        assert nblocks == nbx * nby


def test_ghost_cell_cost_table():
    for n, dim, g1, g2, g3 in read_golden("ghost_cell_cost.txt"):
        # the oracle stores one ghost layer: (bs+2)^d values per block
        t = OracleTree(dim, (n,) * dim, (0,) * dim, (1,) * dim, [DIRICHLET] * (2 * dim), bs=n)
        stored = t.block_field(t.base_level, 0, "v").size
        assert round(stored / n ** dim, 2) == pytest.approx(g1, abs=1e-9)
        for ng, g in ((2, g2), (3, g3)):
            assert round((n + 2 * ng) ** dim / n ** dim, 2) == pytest.approx(g, abs=1e-9)


def _leaf_blocks(t, bs):
    lay = t.leaf_layout()
    blocks = {}
    for lev, i, j, k in lay:
        blocks[(int(lev), int(i) // bs, int(j) // bs, int(k) // bs)] = True
    return list(blocks)


def _boxes(blocks, bs, top):
    out = []
    for lev, bx, by, bz in blocks:
        s = bs * 2 ** (top - lev)
        out.append((lev, np.array([bx * s, by * s, bz * s]), s))
    return out


def _touch(a, b, dim, period):
    (la, oa, sa), (lb, ob, sb) = a, b
    for shift in itertools.product(*[(-1, 0, 1) if period[d] else (0,) for d in range(dim)]):
        ok = True
        for d in range(dim):
            ob_d = ob[d] + shift[d] * period[d]
            if oa[d] > ob_d + sb or ob_d > oa[d] + sa:
                ok = False
                break
        if ok:
            return True
    return False


def _random_predicate(seed, prob):
    rng = np.random.default_rng(seed)
    cache = {}

    def pred(dom, level, origin, bs):
        key = (level, tuple(origin))
        if key not in cache:
            cache[key] = rng.random() < prob
        return cache[key]
    return pred, cache


def _brute_closure(dim, base_blocks, bs, max_refine, cache, periodic):
    """Least tree: refine where the predicate holds (below the top) and wherever a
    leaf touches a leaf two or more levels finer; iterate to a fixed point."""
    leaves = {(0,) + b for b in itertools.product(*[range(n) for n in base_blocks])}
    top = max_refine
    period = [base_blocks[d] * bs * 2 ** top if periodic else 0 for d in range(dim)]

    def children(b):
        lev, idx = b[0], b[1:]
        return {(lev + 1,) + tuple(2 * idx[d] + o[d] for d in range(dim))
                for o in itertools.product((0, 1), repeat=dim)}

    changed = True
    while changed:
        changed = False
        for b in sorted(leaves):
            lev = b[0]
            if lev < top:
                org = tuple(x * bs for x in b[1:]) + (0,) * (3 - dim)
                if cache.get((lev, org), False):
                    leaves.remove(b)
                    leaves |= children(b)
                    changed = True
                    break
        if changed:
            continue
        lst = sorted(leaves)
        boxes = [(b[0], np.array([x * bs * 2 ** (top - b[0]) for x in b[1:]]), bs * 2 ** (top - b[0])) for b in lst]
        for ia, a in enumerate(boxes):
            for ib, bb in enumerate(boxes):
                if bb[0] >= a[0] + 2 and _touch(a, bb, dim, period):
                    leaves.remove(lst[ia])
                    leaves |= children(lst[ia])
                    changed = True
                    break
            if changed:
                break
    return {b if dim == 3 else b + (0,) for b in leaves}


@pytest.mark.parametrize("seed,periodic", [(1, False), (2, True), (3, False), (4, True)])
def test_balance_and_closure_2d(seed, periodic):
    bs, base, max_refine = 2, (4, 4), 3
    pred, cache = _random_predicate(seed, 0.18)
    bc = [PERIODIC if periodic else DIRICHLET] * 4
    t = OracleTree(2, (base[0] * bs, base[1] * bs), (0, 0), (1, 1), bc, bs=bs,
                   max_refine=max_refine, refine=pred)
    got = set(_leaf_blocks(t, bs))
    # every predicate the oracle evaluated is now cached; the brute force uses them
    want = _brute_closure(2, [b for b in base], bs, max_refine, cache, periodic)
    # brute force may visit blocks the oracle did not query; query them too
    for _ in range(3):
        for (lev, bx, by, bz) in list(want):
            if lev < max_refine:
                pred(0, lev, (bx * bs, by * bs, 0), bs)
        want = _brute_closure(2, list(base), bs, max_refine, cache, periodic)
    assert got == want
    # tiling: total leaf volume equals the domain, and balance holds pairwise
    top = max(b[0] for b in got)
    boxes = _boxes(got, bs, top)
    area = sum(s * s for _, _, s in boxes)
    assert area == (base[0] * bs * 2 ** top) * (base[1] * bs * 2 ** top)
    period = [base[d] * bs * 2 ** top if periodic else 0 for d in range(2)]
    for a in boxes:
        for b in boxes:
            if _touch(a, b, 2, period):
                assert abs(a[0] - b[0]) <= 1


def test_balance_3d_corner_refinement():
    # Refining only the block at the origin three times forces its neighbours
    # (across faces, edges and corners) to be refined as well.
    bs = 2

    def pred(dom, level, origin, b):
        return tuple(origin) == (0, 0, 0)
    t = OracleTree(3, (8, 8, 8), (0, 0, 0), (1, 1, 1), [DIRICHLET] * 6, bs=bs, max_refine=3, refine=pred)
    blocks = _leaf_blocks(t, bs)
    top = max(b[0] for b in blocks)
    boxes = _boxes(blocks, bs, top)
    vol = sum(s ** 3 for _, _, s in boxes)
    assert vol == (8 * 2 ** top) ** 3
    for a in boxes:
        for b in boxes:
            if _touch(a, b, 3, [0, 0, 0]):
                assert abs(a[0] - b[0]) <= 1
    assert top == 3


def test_leaf_order_is_level_then_morton():
    bs = 4

    def pred(dom, level, origin, b):
        return level == 0 and origin[0] >= 8
    t = OracleTree(2, (16, 16), (0, 0), (1, 1), [DIRICHLET] * 4, bs=bs, max_refine=1, refine=pred)
    lay = t.leaf_layout()
    # blocks appear contiguously, level ascending, then Morton order of block coords
    keys = []
    for q in range(0, lay.shape[0], bs * bs):
        lev, i, j, _ = lay[q]
        bx, by = i // bs, j // bs
        code = 0
        for bit in range(10):
            code |= ((bx >> bit) & 1) << (2 * bit) | ((by >> bit) & 1) << (2 * bit + 1)
        keys.append((lev, code))
        # x fastest within a block
        blk = lay[q:q + bs * bs]
        assert np.all(blk[:, 1] == i + np.tile(np.arange(bs), bs))
        assert np.all(blk[:, 2] == j + np.repeat(np.arange(bs), bs))
    assert keys == sorted(keys)
