"""The seeded input generators: deterministic, correctly shaped, and matching the
stated recipes (mean removal, eps range, refinement counts)."""
import numpy as np

from oracle import OracleTree
from paper_1901_11370_amd import workloads as W


def _tree(w, d=0, **kw):
    dom = w.domains[d]
    return OracleTree(dom.dim, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bs=w.bs,
                      max_refine=w.max_refine, refine=w.refine, variable_eps=w.variable_eps, **kw)


def test_config2_small_is_seeded_and_mean_free():
    w1, w2 = W.config2(n=32), W.config2(n=32)
    t = _tree(w1)
    lay = t.leaf_layout()
    f1, f2 = w1.rhs(0, lay), w2.rhs(0, lay)
    assert np.array_equal(f1, f2)
    assert abs(f1.mean()) < 1e-15
    assert np.abs(f1).max() > 0.1


def test_config3_literal_rule_refines_only_near_sources():
    w = W.config3(nested=False, base=32)
    t = _tree(w)
    lay = t.leaf_layout()
    assert lay[:, 0].max() >= 1
    f = w.rhs(0, lay)
    assert np.isfinite(f).all()


def test_config4_eps_range():
    w = W.config4(nested=False)
    w.domains[0].base_cells = [32, 32, 32]
    t = _tree(w)
    e = w.eps(0, t.leaf_layout())
    assert e.min() >= 1.0 and e.max() <= 1000.0


def test_config5_fields():
    w = W.config5(sizes=(32, 48))
    for i in range(2):
        t = _tree(w, i)
        lay = t.leaf_layout()
        e = w.eps(i, lay)
        assert e.shape == (t.n_leaf,) and (e > 0).all()
        g = np.log(e) / 0.5
        assert abs(g.std() - 1.0) < 1e-6
        assert w.target(i, lay).max() <= 1e-3
