"""Pins of the oracle's direct sum, reference tree and lists, and DA-FMM:
brute force in high precision on tiny inputs, closed-form uniform-tree counts,
an exact-cover check of the adaptive lists, and the FMM against the direct sum
with geometric decay in the order (Sec. 3.5)."""
import itertools

import mpmath
import numpy as np
import pytest

import oracle
from paper_2508_02626_amd import inputs


def test_direct_matches_mpmath():
    x, q = inputs.uniform(30, 11)
    x[5] = x[3]                      # a coincident pair contributes nothing
    phi, fld = oracle.direct(x, q)
    mpmath.mp.dps = 40
    for i in range(30):
        s = mpmath.mpf(0)
        e = [mpmath.mpf(0)] * 3
        for j in range(30):
            d = [mpmath.mpf(x[i, k]) - mpmath.mpf(x[j, k]) for k in range(3)]
            r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
            if j == i or r2 == 0:
                continue
            r = mpmath.sqrt(r2)
            s += mpmath.mpf(q[j]) / r
            for k in range(3):
                e[k] += mpmath.mpf(q[j]) * d[k] / r ** 3
        assert abs(phi[i] - float(s)) <= 1e-13 * max(1.0, abs(float(s)))
        for k in range(3):
            assert abs(fld[i, k] - float(e[k])) <= 1e-12 * max(1.0, abs(float(e[k])))


def uniform_v_pairs(D):
    """Closed form: V pairs over levels 2..D of the full tree (children of the
    parent's neighbours minus own neighbours), counted per axis."""
    tot = 0
    for l in range(2, D + 1):
        n = 2 ** l
        # per axis: pairs (i, j) with |i - j| <= 1 at parent level and |i-j| > 1
        par = sum(1 for i in range(n) for j in range(n) if abs(i // 2 - j // 2) <= 1)
        near = sum(1 for i in range(n) for j in range(n) if abs(i - j) <= 1)
        tot += par ** 3 - near ** 3
    return tot


@pytest.mark.parametrize("D", [2, 3, 4])
def test_uniform_tree_counts(D):
    x, q = inputs.uniform(3000, 0)
    t = oracle.Tree(x, root=[0, 0, 0, 1], uniform_depth=D)
    assert t.nboxes == sum(8 ** l for l in range(D + 1))
    n = 2 ** D
    assert t.nU == (3 * n - 2) ** 3
    assert t.nV == uniform_v_pairs(D)
    assert t.nW == 0 and t.nX == 0
    e = t.export()
    lv = e["level"]
    # interior boxes have 189 V entries; 316 distinct offsets overall
    V_off, V_src, mort = e["V_off"], e["V_src"], e["morton"]
    def coords(code, l):
        c = [0, 0, 0]
        for b in range(l):
            c[0] |= ((int(code) >> (3 * b + 2)) & 1) << b
            c[1] |= ((int(code) >> (3 * b + 1)) & 1) << b
            c[2] |= ((int(code) >> (3 * b)) & 1) << b
        return c
    offs = set()
    maxv = 0
    for b in range(t.nboxes):
        cnt = V_off[b + 1] - V_off[b]
        maxv = max(maxv, cnt)
        cb = coords(mort[b], lv[b])
        for s in V_src[V_off[b]:V_off[b + 1]]:
            cs = coords(mort[s], lv[s])
            offs.add(tuple(cb[k] - cs[k] for k in range(3)))
    if D >= 3:
        assert maxv == 189
        assert len(offs) == 316


def test_config1_sizes():
    x, q = inputs.uniform(2000, 0)
    t = oracle.Tree(x, root=[0, 0, 0, 1], uniform_depth=3)
    assert (t.nboxes, t.nV, t.nU) == (585, 56448, 10648)


def _ancestors(parent, b):
    out = [b]
    while parent[b] >= 0:
        b = parent[b]
        out.append(b)
    return out


@pytest.mark.parametrize("gen,n,s", [("plummer", 3000, 16), ("clusters", 2500, 10), ("uniform", 1500, 8)])
def test_adaptive_lists_cover_every_pair_once(gen, n, s):
    """Every (target leaf, source leaf) pair is handled exactly once by
    U, by V between ancestors, by W (M2P) or by X (P2L)."""
    x, q = getattr(inputs, gen)(n, 3)
    t = oracle.Tree(x, leaf_size=s)
    e = t.export()
    par, nch = e["parent"], e["nchild"]
    leaves = [b for b in range(t.nboxes) if nch[b] == 0]
    anc = {b: set(_ancestors(par, b)) for b in range(t.nboxes)}
    def lst(k, b):
        return set(e[k + "_src"][e[k + "_off"][b]:e[k + "_off"][b + 1]].tolist())
    V = {b: lst("V", b) for b in range(t.nboxes)}
    X = {b: lst("X", b) for b in range(t.nboxes)}
    for B in leaves:
        U, W = lst("U", B), lst("W", B)
        assert B in U
        xs = set().union(*[X[A] for A in anc[B]])
        vs = [(A, C) for A in anc[B] for C in V[A]]
        for C in leaves:
            cnt = (C in U) + (C in xs)
            cnt += sum(1 for A2 in anc[C] if A2 in W)
            cnt += sum(1 for (A, C2) in vs if C2 in anc[C])
            assert cnt == 1, (B, C, cnt)
    # the counts of particles per leaf respect the leaf size or the depth cap
    for b in leaves:
        assert e["count"][b] <= s or e["level"][b] == t.key_depth
    assert e["count"][0] == n and sorted(e["perm"].tolist()) == list(range(n))


def test_fmm_memo_equals_full_composition():
    x, q = inputs.uniform(600, 0)
    t = oracle.Tree(x, root=[0, 0, 0, 1], uniform_depth=3)
    a, fa = t.fmm(4, q, memo=True)
    b, fb = t.fmm(4, q, memo=False)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    assert np.max(np.abs(fa - fb)) <= 1e-12 * np.max(np.abs(fa))


def test_fmm_shallow_tree_is_direct():
    """Depth <= 1: every leaf is adjacent to every other, so the FMM is the direct sum."""
    x, q = inputs.uniform(300, 1)
    d, fd = oracle.direct(x, q)
    for D in (0, 1):
        t = oracle.Tree(x, root=[0, 0, 0, 1], uniform_depth=D)
        a, fa = t.fmm(3, q)
        assert np.allclose(a, d, rtol=1e-13, atol=1e-13 * np.abs(d).max())
        assert np.allclose(fa, fd, rtol=1e-12, atol=1e-12 * np.abs(fd).max())


def test_fmm_config1_error_decays_with_order():
    """Sec. 3.5: the error against the exact potential falls steadily with p."""
    x, q = inputs.uniform(2000, 0)
    t = oracle.Tree(x, root=[0, 0, 0, 1], uniform_depth=3)
    d, fd = oracle.direct(x, q)
    errs = []
    for p in (2, 4, 6, 8):
        a, fa = t.fmm(p, q)
        errs.append(np.linalg.norm(a - d) / np.linalg.norm(d))
    errs = np.array(errs)
    assert np.all(errs[1:] < 0.4 * errs[:-1]), errs
    assert errs[-1] < 5e-5


def test_fmm_adaptive_against_direct():
    x, q = inputs.plummer(6000, 2)
    t = oracle.Tree(x, leaf_size=32)
    assert t.nW > 0 and t.nX > 0
    d, fd = oracle.direct(x, q)
    errs = []
    for p in (3, 6):
        a, fa = t.fmm(p, q)
        errs.append(np.linalg.norm(a - d) / np.linalg.norm(d))
    assert errs[1] < 0.1 * errs[0] and errs[1] < 1e-3, errs
