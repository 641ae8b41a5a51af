"""GPU octree and interaction lists against the oracle, bit for bit (Sec. 1
recursive subdivision, Sec. 3.5 leaf size s, Sec. 3.4 interaction lists)."""
import numpy as np
import pytest

from paper_2508_02626_amd import inputs
from gpu_util import TREE_KEYS, gpu_solve, oracle_tree, say, to_dev

pytestmark = pytest.mark.gpu


def _cases():
    c = []
    c.append(("config1_uniform_d3", lambda: inputs.uniform(2000, 0), dict(uniform_depth=3, root=[0, 0, 0, 1])))
    c.append(("uniform_d5_1e5", lambda: inputs.uniform(100_000, 1), dict(uniform_depth=5, root=[0, 0, 0, 1])))
    c.append(("uniform_d4_bbox", lambda: inputs.uniform(30_000, 4), dict(uniform_depth=4)))
    # shallow and sparse uniform trees: no level >= 2 (no V lists), and many empty leaves
    c.append(("uniform_d0", lambda: inputs.uniform(50, 11), dict(uniform_depth=0, root=[0, 0, 0, 1])))
    c.append(("uniform_d1", lambda: inputs.uniform(300, 12), dict(uniform_depth=1, root=[0, 0, 0, 1])))
    c.append(("uniform_d4_sparse", lambda: inputs.uniform(40, 13), dict(uniform_depth=4, root=[0, 0, 0, 1])))
    c.append(("plummer_5e4_s64", lambda: inputs.plummer(50_000, 2), dict(leaf_size=64)))
    c.append(("plummer_2e4_s16", lambda: inputs.plummer(20_000, 5), dict(leaf_size=16)))
    c.append(("clusters_3e4_s32", lambda: inputs.clusters(30_000, 6), dict(leaf_size=32)))
    c.append(("gaussian_2e4_s40", lambda: inputs.gaussian(20_000, 7), dict(leaf_size=40)))
    c.append(("ragged_997_s7", lambda: inputs.uniform(997, 8), dict(leaf_size=7)))
    c.append(("n1", lambda: (np.array([[0.3, 0.2, 0.1]]), np.array([1.0])), dict(leaf_size=4)))
    c.append(("n2_coincident", lambda: (np.array([[0.5, 0.5, 0.5]] * 2), np.array([1.0, -2.0])), dict(leaf_size=1)))
    c.append(("identical_200_cap", lambda: (np.tile([[0.1, 0.7, 0.3]], (200, 1)), np.ones(200)),
              dict(leaf_size=8, max_depth=5)))
    c.append(("plummer_maxdepth4", lambda: inputs.plummer(5000, 9), dict(leaf_size=4, max_depth=4)))

    def boundary():
        rng = np.random.default_rng(3)
        x = rng.integers(0, 5, (500, 3)) / 4.0  # on box faces and at 0 and 1
        return x, rng.uniform(-1, 1, 500)
    c.append(("boundary_points", boundary, dict(uniform_depth=3, root=[0, 0, 0, 1])))
    c.append(("boundary_adaptive", boundary, dict(leaf_size=3)))
    return c


@pytest.mark.parametrize("name,gen,kw", _cases(), ids=[c[0] for c in _cases()])
def test_tree_bit_exact(name, gen, kw):
    from paper_2508_02626_amd import fmm
    x, q = gen()
    say("tree case", name, "n", len(q), kw)
    pl = fmm.Plan(to_dev(x), 3, **kw)
    g = pl.export_tree()
    t = oracle_tree(x, **kw)
    o = t.export()
    assert np.array_equal(g["root"], t.root)
    s = pl.sizes()
    assert (s["boxes"], s["U"], s["V"], s["W"], s["X"], s["depth"]) == \
        (t.nboxes, t.nU, t.nV, t.nW, t.nX, t.depth)
    for k in TREE_KEYS:
        assert g[k].shape == o[k].shape, k
        assert np.array_equal(g[k].astype(np.int64), o[k].astype(np.int64)), k
    pl.close()
