"""Pins of the oracle's DA-FMM operators (Sec. 2) against facts the paper and
the mathematics fix: the exact low orders of P2M (Sec. 3.1), the Legendre
generating function, harmonicity, exactness of M2M, the point-charge special
case of M2L, the bit-identical top degree of L2L (Sec. 3.3), polynomial
invariance of L2L, brute force against the direct sum with geometric decay in
the order, and finite differences for fields."""
import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle

EXP = {p: oracle.exponents(p) for p in range(0, 13)}


def mono(p, y):
    e = EXP[p]
    y = np.asarray(y, dtype=float)
    return np.prod(y[None, :] ** e, axis=1)


def charges(n, seed, half=0.5, center=(0, 0, 0)):
    rng = np.random.default_rng(seed)
    x = np.asarray(center) + rng.uniform(-half, half, (n, 3))
    q = rng.uniform(-1, 1, n)
    return x, q


def test_p2m_orders_0_and_1_exact():
    """Sec. 3.1: the constant part and all first-order coefficients agree exactly:
    M_0 = sum q, M_{e_k} = sum q y_k."""
    x, q = charges(50, 1)
    M = oracle.p2m(5, x, q, [0.1, -0.2, 0.05])
    y = x - np.array([0.1, -0.2, 0.05])
    assert abs(M[0] - q.sum()) <= 1e-14 * np.abs(q).sum()
    for k in range(3):
        assert abs(M[1 + k] - (q * y[:, k]).sum()) <= 1e-14 * np.abs(q).sum()


@pytest.mark.parametrize("p", [4, 8])
def test_p2m_is_legendre_generating_function(p):
    """(1 - 2 y.d + y^2 d^2)^(-1/2) = sum_n |y|^n |d|^n P_n(cos): the degree-n part
    of P2M for one unit charge, at a unit vector u, is |y|^n P_n(y_hat . u)."""
    y = np.array([0.3, -0.2, 0.45])
    M = oracle.p2m(p, y[None, :], np.ones(1), [0, 0, 0])
    rng = np.random.default_rng(2)
    deg = EXP[p].sum(axis=1)
    for _ in range(5):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        m = mono(p, u)
        for n in range(p + 1):
            got = np.sum((M * m)[deg == n])
            ref = np.linalg.norm(y) ** n * eval_legendre(n, y @ u / np.linalg.norm(y))
            assert abs(got - ref) <= 1e-13


def laplacian(p, v):
    dxx = oracle.da_op("dx", p, oracle.da_op("dx", p, v))
    dyy = oracle.da_op("dy", p, oracle.da_op("dy", p, v))
    dzz = oracle.da_op("dz", p, oracle.da_op("dz", p, v))
    return dxx + dyy + dzz


def test_p2m_degrees_are_harmonic():
    x, q = charges(20, 3)
    M = oracle.p2m(8, x, q, [0, 0, 0])
    assert np.max(np.abs(laplacian(8, M))) <= 1e-12 * np.max(np.abs(M))


@pytest.mark.parametrize("p", [4, 6, 8, 10])
def test_m2m_is_exact(p):
    """M2M of a child's P2M equals P2M about the parent centre (the map M1 of
    Sec. 2.2 re-expands the truncated multipole without loss)."""
    h = 0.5
    cc = np.array([0.25, -0.25, 0.25]) * h * 2
    pc = np.zeros(3)
    x, q = charges(40, 4, half=h / 2, center=cc)
    Mc = oracle.p2m(p, x, q, cc)
    Mp = oracle.m2m(p, cc, pc, Mc)
    ref = oracle.p2m(p, x, q, pc)
    assert abs(Mp[0] - Mc[0]) <= 1e-15 * abs(Mc[0])     # order 0 conserved
    assert np.max(np.abs(Mp - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_m2l_point_charge_equals_p2l():
    """A charge at the source centre has M = q e_0; its local expansion is then
    the Taylor expansion of q/|r0 + d'| (Eq. P2L)."""
    p = 8
    M = np.zeros(oracle.ncoef(p))
    M[0] = 0.7
    sc, tc = np.array([0.1, 0.2, -0.3]), np.array([2.1, -0.8, 0.7])
    L = oracle.m2l(p, sc, tc, M)
    ref = oracle.p2l(p, sc[None, :], np.array([0.7]), tc)
    assert np.max(np.abs(L - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_m2l_far_field_decays_geometrically():
    """L2P(M2L(P2M(S))) against the direct sum for boxes one box apart: the error
    falls by a steady factor with the order."""
    h = 1.0
    sc, tc = np.zeros(3), np.array([2.0, 1.0, 0.0])
    xs, qs = charges(60, 5, half=h / 2, center=sc)
    xt, _ = charges(30, 6, half=h / 2, center=tc)
    allx = np.vstack([xs, xt])
    allq = np.concatenate([qs, np.zeros(len(xt))])
    ref, fref = oracle.direct(allx, allq, np.arange(60, 90))
    errs = []
    for p in (2, 4, 6, 8, 10):
        L = oracle.m2l(p, sc, tc, oracle.p2m(p, xs, qs, sc))
        phi, fld = oracle.l2p(p, tc, L, xt)
        errs.append(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
    errs = np.array(errs)
    assert np.all(errs[1:] < 0.6 * errs[:-1]), errs
    assert errs[-1] < 1e-4


def test_l2l_top_degree_bit_identical_and_polynomial_invariant():
    """Sec. 3.3: a linear shift changes only lower-order terms, so the highest
    degree is reproduced exactly; and L2P(L2L(L), x) = L2P(L, x)."""
    p = 7
    rng = np.random.default_rng(7)
    L = rng.normal(size=oracle.ncoef(p))
    pc, cc = np.array([0.0, 0.0, 0.0]), np.array([0.25, -0.25, 0.25])
    L2 = oracle.l2l(p, pc, cc, L)
    top = EXP[p].sum(axis=1) == p
    assert np.array_equal(L2[top], L[top])
    pts = cc + rng.uniform(-0.25, 0.25, (10, 3))
    a, fa = oracle.l2p(p, pc, L, pts)
    b, fb = oracle.l2p(p, cc, L2, pts)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())
    assert np.allclose(fa, fb, rtol=1e-11, atol=1e-11 * np.abs(fa).max())


def test_p2l_and_m2p_against_direct():
    p = 10
    xs, qs = charges(40, 8, half=0.5, center=(0, 0, 0))
    tc = np.array([0.0, 3.0, 0.0])
    xt, _ = charges(20, 9, half=0.5, center=tc)
    allx = np.vstack([xs, xt])
    allq = np.concatenate([qs, np.zeros(20)])
    ref, fref = oracle.direct(allx, allq, np.arange(40, 60))
    phi, fld = oracle.l2p(p, tc, oracle.p2l(p, xs, qs, tc), xt)
    assert np.linalg.norm(phi - ref) / np.linalg.norm(ref) < 1e-4
    assert np.linalg.norm(fld - fref) / np.linalg.norm(fref) < 1e-3
    phi, fld = oracle.m2p(p, np.zeros(3), oracle.p2m(p, xs, qs, np.zeros(3)), xt)
    assert np.linalg.norm(phi - ref) / np.linalg.norm(ref) < 1e-4
    assert np.linalg.norm(fld - fref) / np.linalg.norm(fref) < 1e-3


@pytest.mark.parametrize("which", ["l2p", "m2p"])
def test_fields_match_finite_differences(which):
    p = 6
    rng = np.random.default_rng(10)
    c = np.array([0.2, -0.1, 0.3])
    if which == "l2p":
        v = oracle.p2l(p, np.array([[3.0, 0.5, -1.0]]), np.array([1.0]), c)
        pts = c + rng.uniform(-0.2, 0.2, (5, 3))
        fn = oracle.l2p
    else:
        v = oracle.p2m(p, c + rng.uniform(-0.2, 0.2, (6, 3)), rng.uniform(-1, 1, 6), c)
        pts = c + np.array([[2.0, 0.3, -0.5]]) + rng.uniform(-0.2, 0.2, (5, 3))
        fn = oracle.m2p
    _, fld = fn(p, c, v, pts)
    eps = 1e-5
    for k in range(3):
        dp = np.zeros(3)
        dp[k] = eps
        a, _ = fn(p, c, v, pts + dp)
        b, _ = fn(p, c, v, pts - dp)
        fd = -(a - b) / (2 * eps)
        assert np.allclose(fld[:, k], fd, rtol=1e-7, atol=1e-8)
