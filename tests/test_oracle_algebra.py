"""Pins of the oracle's truncated power series algebra (App. A) against values
the paper prints (Table 1) and against exact symbolic series (sympy)."""
import os
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_inv_r_111.txt")


def _table1():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    return [tuple(int(v) for v in r[:3]) for r in rows], np.array([float(r[3]) for r in rows])


def test_table1_monomial_order():
    exps, _ = _table1()
    assert [tuple(e) for e in oracle.exponents(2)] == exps


def test_table1_values():
    """Table 1 (Sec. 3): DA of 1/r at (1,1,1), order 2, to the printed digits."""
    _, vals = _table1()
    got = oracle.da_inv_r(2, [1.0, 1.0, 1.0])
    for g, v in zip(got, vals):
        if abs(v) < 1e-16:          # printed 8.0e-18 is round-off of an exact 0
            assert abs(g) < 1e-16
        else:
            assert abs(g - v) <= 2e-16 * abs(v) + 1e-17


X, Y, Z = sp.symbols("x y z")


def _sympy_taylor(expr, point, p):
    """Taylor coefficients (1/J! d^J f) of expr about point, in oracle order."""
    out = []
    for (i, j, k) in oracle.exponents(p):
        d = sp.diff(expr, X, i, Y, j, Z, k) if i + j + k else expr
        val = d.subs({X: point[0], Y: point[1], Z: point[2]})
        out.append(float(val / (sp.factorial(i) * sp.factorial(j) * sp.factorial(k))))
    return np.array(out)


@pytest.mark.parametrize("pt", [(1, 1, 1), (2, -1, 3), (Fraction(1, 2), Fraction(-3, 4), 2)])
def test_inv_r_matches_exact_derivatives(pt):
    p = 5
    ref = _sympy_taylor(1 / sp.sqrt(X ** 2 + Y ** 2 + Z ** 2),
                        [sp.Rational(v.numerator, v.denominator) if isinstance(v, Fraction) else v for v in pt], p)
    got = oracle.da_inv_r(p, [float(v) for v in pt])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-14 * scale


def _da_from_poly(poly, p):
    """DA vector (order p) of a sympy polynomial in d1,d2,d3 = X,Y,Z."""
    P = sp.Poly(sp.expand(poly), X, Y, Z)
    v = np.zeros(oracle.ncoef(p))
    idx = {tuple(e): n for n, e in enumerate(oracle.exponents(p))}
    for (i, j, k), c in P.terms():
        if i + j + k <= p:
            v[idx[(i, j, k)]] = float(c)
    return v


def test_product_truncates():
    p = 3
    a = 1 + X - 2 * Y * Z + Z ** 3
    b = 2 - X ** 2 + 3 * Y
    got = oracle.da_op("mul", p, _da_from_poly(a, p), _da_from_poly(b, p))
    full = sp.Poly(sp.expand(a * b), X, Y, Z)
    trunc = sum(c * X ** i * Y ** j * Z ** k for (i, j, k), c in full.terms() if i + j + k <= p)
    assert np.allclose(got, _da_from_poly(trunc, p), rtol=0, atol=1e-15)


@pytest.mark.parametrize("op,fn", [("inv", lambda e: 1 / e), ("sqrt", sp.sqrt)])
def test_inverse_and_root_match_series(op, fn):
    """App. A: inverse and roots of a non-infinitely-small element, order by order."""
    p = 6
    a = sp.Rational(3, 2) + X - sp.Rational(1, 3) * Y + 2 * X * Z - Z ** 2 / 5
    ref = _sympy_taylor(fn(a), (0, 0, 0), p)
    got = oracle.da_op(op, p, _da_from_poly(a, p))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_derivation():
    """Eq. dev: d/dx_v of a polynomial."""
    p = 4
    a = 1 + 3 * X ** 2 * Y - Y * Z ** 3 + X * Y * Z
    for op, v in (("dx", X), ("dy", Y), ("dz", Z)):
        got = oracle.da_op(op, p, _da_from_poly(a, p))
        assert np.allclose(got, _da_from_poly(sp.diff(a, v), p), atol=1e-15)


def test_composition_is_substitution():
    """f o g for polynomials whose composite stays within the order."""
    p = 4
    f = 1 + X - 2 * Y ** 2 + X * Y * Z
    g = [sp.Rational(1, 2) + Y, X - Z, 2 * X]
    got = oracle.da_compose(2 * 0 + 4, _da_from_poly(f, p), 4,
                            np.concatenate([_da_from_poly(gi, 4) for gi in g]))
    ref = sp.expand(f.subs({X: g[0], Y: g[1], Z: g[2]}, simultaneous=True))
    assert np.allclose(got, _da_from_poly(ref, 4), atol=1e-14)
