"""The work counts behind bench.py's roofline figures, against independent
enumerations: the parity-class sizes of the harmonic (Coulomb) and Cartesian
(softened) components, and the sign-class M2L work of small trees recounted
pair by pair from the V lists (every (row, column) monomial pair a class's
contraction keeps, plus the member butterflies)."""
import os
import sys

import numpy as np
import pytest

import oracle

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def parity(i, j, k):
    return (i & 1) << 2 | (j & 1) << 1 | (k & 1)


def cart_monomials(p):
    return [(i, j, k) for i in range(p + 1) for j in range(p + 1 - i) for k in range(p + 1 - i - j)]


def harm_monomials(p):
    # folded harmonic components: exponents (i, j, kz) with kz in {0, 1}, i + j + kz <= p
    return [(i, j, kz) for kz in (0, 1) for i in range(p + 1) for j in range(p + 1 - i - kz)]


@pytest.mark.parametrize("p", [0, 1, 4, 8, 10, 14])
def test_class_sizes(p):
    cart = [0] * 8
    for g in cart_monomials(p):
        cart[parity(*g)] += 1
    assert bench.cart_class_counts(p) == cart
    assert sum(cart) == (p + 1) * (p + 2) * (p + 3) // 6
    harm = [0] * 8
    for g in harm_monomials(p):
        harm[parity(*g)] += 1
    assert bench.sym_class_counts(p) == harm
    assert sum(harm) == (p + 1) ** 2


def brute_work(t, p, cartesian):
    """Sum over targets and over the distinct |k| of their V pairs of 2 x the
    monomial pairs (a, b) whose parity difference avoids the zero axes of |k|,
    plus |P| 2^|P| additions per column (P: axes with |k| in {1, 2})."""
    mons = cart_monomials(p) if cartesian else harm_monomials(p)
    par = [parity(*g) for g in mons]
    vo, vs = t["V_off"], t["V_src"]
    lev, mor = t["level"], t["morton"]

    def cell(b):
        c = [0, 0, 0]
        for bit in range(int(lev[b])):
            for d in range(3):
                c[d] |= ((int(mor[b]) >> (3 * bit + 2 - d)) & 1) << bit
        return c

    total = 0.0
    for tg in range(len(vo) - 1):
        classes = set()
        ct = cell(tg)
        for e in range(vo[tg], vo[tg + 1]):
            cs = cell(int(vs[e]))
            classes.add(tuple(abs(ct[d] - cs[d]) for d in range(3)))
        for a in classes:
            zero = sum(4 >> d for d in range(3) if a[d] == 0)
            pairs = sum(1 for x in par for y in par if not ((x ^ y) & zero))
            npair = sum(1 for d in range(3) if a[d] in (1, 2))
            total += 2.0 * pairs + npair * 2 ** npair * len(mons)
    return total


@pytest.mark.parametrize("cartesian,p,kw", [(True, 4, dict(uniform_depth=3, root=[0, 0, 0, 1.0])),
                                            (True, 3, dict(leaf_size=10)),
                                            (False, 6, dict(uniform_depth=3, root=[0, 0, 0, 1.0])),
                                            (False, 5, dict(leaf_size=10))])
def test_m2l_work_matches_pair_count(cartesian, p, kw):
    rng = np.random.default_rng(3)
    if "leaf_size" in kw:
        c = rng.uniform(0.2, 0.8, (3, 3))
        x = c[rng.integers(0, 3, 700)] + 0.06 * rng.normal(size=(700, 3))
    else:
        x = rng.uniform(0, 1, (600, 3))
    t = oracle.Tree(x, **kw).export()
    flops, nv = bench.m2l_work(t, p, cartesian=cartesian)
    assert nv == len(t["V_src"]) and nv > 0
    assert flops == pytest.approx(brute_work(t, p, cartesian), rel=1e-12)
