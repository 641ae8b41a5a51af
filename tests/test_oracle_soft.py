"""Pins of the oracle's softened Coulomb kernel K(x) = 1/sqrt(|x|^2 + eps^2)
(the second non-oscillatory kernel; DA-based formulations extend to such
kernels, closing remark of Sec. 3.4) against facts fixed by the paper and the
mathematics: Table 1 at eps = 0, exact symbolic Taylor coefficients, a
40-digit direct sum, the Coulomb oracle (an independent construction through
Eq. P2M's inversion) at eps = 0, exactness of the moment M2M, polynomial
invariance of L2L, geometric decay of M2L/P2L/M2P/FMM errors with the order,
trees without far field, finite differences for the fields, the reflection
symmetry of K's derivatives and the sign-class decomposition of the M2L
(one contraction per class of offsets, members combined by a Walsh-Hadamard
transform) against the oracle's own M2L."""
import os

import mpmath
import numpy as np
import pytest
import sympy as sp

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_inv_r_111.txt")
X, Y, Z = sp.symbols("x y z")


def pts(n, seed, half=0.5, center=(0, 0, 0)):
    rng = np.random.default_rng(seed)
    return np.asarray(center) + rng.uniform(-half, half, (n, 3)), rng.uniform(-1, 1, n)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def test_taylor_at_eps0_is_table1():
    """eps = 0: the kernel is 1/r, and its DA vector at (1,1,1) to order 2 is
    the one Table 1 prints."""
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    vals = np.array([float(r[3]) for r in rows])
    got = oracle.soft_taylor(2, [1.0, 1.0, 1.0], 0.0)
    for g, v in zip(got, vals):
        assert abs(g - v) <= 2e-16 * abs(v) + 1e-16


@pytest.mark.parametrize("x0,eps", [((0.3, -0.7, 1.1), 0.4), ((1.5, 0.2, -0.4), 0.05), ((0.0, 0.0, 0.0), 0.8)])
def test_taylor_matches_sympy(x0, eps):
    """Coefficients d^g K(x0) / g! against exact symbolic derivatives (order 5),
    including the centre of the kernel (x0 = 0, finite only for eps > 0)."""
    p = 5
    e = sp.Rational(str(eps))
    f = 1 / sp.sqrt(X ** 2 + Y ** 2 + Z ** 2 + e ** 2)
    got = oracle.soft_taylor(p, x0, eps)
    pt = {X: sp.Rational(str(x0[0])), Y: sp.Rational(str(x0[1])), Z: sp.Rational(str(x0[2]))}
    for idx, (i, j, k) in enumerate(oracle.exponents(p)):
        d = sp.diff(f, X, i, Y, j, Z, k) if i + j + k else f
        ref = float(d.subs(pt)) / (sp.factorial(i) * sp.factorial(j) * sp.factorial(k))
        assert abs(got[idx] - ref) <= 1e-13 * max(1.0, abs(ref)), (i, j, k)


def test_direct_soft_matches_mpmath():
    """The O(N^2) sum against 40-digit arithmetic, with a coincident pair (which
    interacts through q/eps when eps > 0) and eps = 0 (where it does not)."""
    x, q = pts(40, 3)
    x[7] = x[3]
    mpmath.mp.dps = 40
    for eps in (0.05, 0.0):
        phi, fld = oracle.direct_soft(x, q, eps)
        for i in (0, 3, 7, 25):
            ph = mpmath.mpf(0)
            E = [mpmath.mpf(0)] * 3
            for j in range(len(q)):
                if j == i:
                    continue
                d = [mpmath.mpf(x[i, k]) - mpmath.mpf(x[j, k]) for k in range(3)]
                s2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + mpmath.mpf(eps) ** 2
                if s2 == 0:
                    continue
                ph += mpmath.mpf(q[j]) / mpmath.sqrt(s2)
                for k in range(3):
                    E[k] += mpmath.mpf(q[j]) * d[k] / s2 ** mpmath.mpf(1.5)
            assert abs(phi[i] - float(ph)) <= 1e-14 * abs(float(ph)) + 1e-14
            for k in range(3):
                assert abs(fld[i, k] - float(E[k])) <= 1e-13 * max(1.0, abs(float(E[k])))


@pytest.mark.parametrize("p,kw", [(6, dict(uniform_depth=3)), (5, dict(leaf_size=12))])
def test_fmm_at_eps0_equals_coulomb_oracle(p, kw):
    """At eps = 0 the softened FMM (moments, Taylor coefficients from the DA)
    must reproduce the Coulomb DA-FMM of Sec. 2 (inversion, DA composition):
    the same truncated expansions built two different ways."""
    rng = np.random.default_rng(11)
    if "uniform_depth" in kw:
        x = rng.uniform(0, 1, (1500, 3))
        root = [0.0, 0.0, 0.0, 1.0]
    else:
        c = rng.uniform(0.2, 0.8, (4, 3))
        x = c[rng.integers(0, 4, 800)] + 0.05 * rng.normal(size=(800, 3))
        root = None
    q = rng.uniform(-1, 1, len(x))
    t = oracle.Tree(x, root=root, **kw)
    assert t.nV > 0 and (("uniform_depth" in kw) or (t.nW > 0 and t.nX > 0))
    phs, fs = t.fmm_soft(p, q, 0.0)
    phc, fc = t.fmm(p, q)
    assert rel(phs, phc) <= 1e-12
    assert rel(fs, fc) <= 1e-12


def test_fmm_without_far_field_is_direct():
    """Trees of depth <= 1 have no V, W or X lists: the FMM is the direct sum."""
    x, q = pts(300, 5, center=(0.5, 0.5, 0.5))
    for depth in (0, 1):
        t = oracle.Tree(x, root=[0, 0, 0, 1.0], uniform_depth=depth)
        phi, fld = t.fmm_soft(6, q, 0.03)
        pd, fd = oracle.direct_soft(x, q, 0.03)
        assert rel(phi, pd) <= 1e-14 and rel(fld, fd) <= 1e-14


@pytest.mark.parametrize("kw", [dict(uniform_depth=3), dict(leaf_size=16)])
def test_fmm_error_decays_with_order(kw):
    """Against the softened direct sum the error falls geometrically with p."""
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 1, (1200, 3))
    q = rng.uniform(-1, 1, 1200)
    eps = 0.02
    t = oracle.Tree(x, root=[0, 0, 0, 1.0], **kw)
    pd, fd = oracle.direct_soft(x, q, eps)
    errs = [rel(t.fmm_soft(p, q, eps)[0], pd) for p in (2, 4, 6, 8)]
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 2e-4


def test_m2m_is_exact_for_moments():
    """Moments of the child shifted to the parent equal the parent's moments
    of the same charges (a binomial identity: exact up to rounding)."""
    x, q = pts(60, 2, half=0.25, center=(0.25, -0.25, 0.25))
    for p in (3, 8):
        Mc = oracle.soft_p2m(p, x, q, [0.25, -0.25, 0.25])
        Mp = oracle.soft_m2m(p, [0.25, -0.25, 0.25], [0, 0, 0], Mc)
        ref = oracle.soft_p2m(p, x, q, [0, 0, 0])
        assert np.max(np.abs(Mp - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_l2l_keeps_the_polynomial():
    """L2L re-expands a polynomial of degree p exactly about another centre."""
    p = 7
    rng = np.random.default_rng(4)
    L = rng.normal(size=oracle.ncoef(p))
    e = oracle.exponents(p)
    c0, c1 = np.array([0.0, 0.0, 0.0]), np.array([0.25, -0.25, 0.25])
    L1 = oracle.soft_l2l(p, c0, c1, L)
    for xx in rng.uniform(-0.5, 0.5, (5, 3)):
        v0 = np.sum(L * np.prod((xx - c0)[None, :] ** e, axis=1))
        v1 = np.sum(L1 * np.prod((xx - c1)[None, :] ** e, axis=1))
        assert abs(v0 - v1) <= 1e-13 * np.sum(np.abs(L))


def test_m2l_and_p2l_converge_to_the_direct_sum():
    """Charges in a source box, local expansion at a well-separated target box:
    M2L(P2M) and P2L evaluated near the target centre approach the direct sum
    with geometric decay, and agree exactly for a charge at the source centre."""
    eps = 0.1
    x, q = pts(30, 6, half=0.5)
    cs, ct = np.zeros(3), np.array([2.0, 1.0, -2.0])
    y = ct + np.random.default_rng(7).uniform(-0.3, 0.3, (6, 3))
    ref = np.array([np.sum(q / np.sqrt(np.sum((yy - x) ** 2, axis=1) + eps ** 2)) for yy in y])
    errs = {"m2l": [], "p2l": []}
    for p in (2, 4, 6, 8):
        e = oracle.exponents(p)
        M = oracle.soft_p2m(p, x, q, cs)
        for name, L in (("m2l", oracle.soft_m2l(p, eps, cs, ct, M)), ("p2l", oracle.soft_p2l(p, eps, x, q, ct))):
            got = np.array([np.sum(L * np.prod((yy - ct)[None, :] ** e, axis=1)) for yy in y])
            errs[name].append(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    for v in errs.values():
        assert all(b < 0.6 * a for a, b in zip(v, v[1:])), errs
        assert v[-1] < 1e-4, errs
    one = np.array([[0.0, 0.0, 0.0]])
    La = oracle.soft_m2l(6, eps, cs, ct, oracle.soft_p2m(6, one, np.ones(1), cs))
    Lb = oracle.soft_p2l(6, eps, one, np.ones(1), ct)
    assert np.max(np.abs(La - Lb)) <= 1e-15 * np.max(np.abs(Lb))


def test_fmm_fields_are_gradients():
    """The field the FMM returns is minus the gradient of the potential it
    returns (central differences inside a leaf, away from its faces)."""
    rng = np.random.default_rng(9)
    x = rng.uniform(0.05, 0.95, (400, 3))
    q = rng.uniform(-1, 1, 400)
    eps = 0.05
    root = [0.0, 0.0, 0.0, 1.0]
    t = oracle.Tree(x, root=root, uniform_depth=2)
    i = 17
    phi, fld = t.fmm_soft(5, q, eps)
    hstep = 1e-5
    for k in range(3):
        xp, xm = x.copy(), x.copy()
        xp[i, k] += hstep
        xm[i, k] -= hstep
        # move particle i as a target only: the sum over sources excludes j = i
        tp = oracle.Tree(xp, root=root, uniform_depth=2)
        tm = oracle.Tree(xm, root=root, uniform_depth=2)
        qz = q.copy()
        qz[i] = 0.0  # its own charge must not move with it
        php = tp.fmm_soft(5, qz, eps)[0][i]
        phm = tm.fmm_soft(5, qz, eps)[0][i]
        fd = -(php - phm) / (2 * hstep)
        assert abs(fd - fld[i, k]) <= 1e-6 * max(1.0, abs(fld[i, k]))


def test_derivatives_change_sign_with_odd_exponents():
    """K is even in every coordinate: the Taylor coefficient of exponent g at
    the offset with some axes negated is the one at k times (-1)^(g on those
    axes) (the reflection the GPU's sign-class M2L rests on)."""
    p, eps = 6, 0.3
    e = oracle.exponents(p)
    k = np.array([2.0, -1.0, 3.0])
    base = oracle.soft_taylor(p, k, eps)
    for m in range(8):
        s = np.array([-1.0 if (m >> (2 - d)) & 1 else 1.0 for d in range(3)])
        got = oracle.soft_taylor(p, s * k, eps)
        sign = np.prod(s[None, :] ** e, axis=1)
        assert np.allclose(got, sign * base, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("rep", [(2, 1, 3), (0, 2, 1), (3, 0, 0)])
def test_sign_class_contraction_equals_member_sum(rep):
    """Sum over the members of a sign class (offsets s o k, s over the signs
    of the non-zero axes) of the oracle's M2L equals one contraction with the
    representative's matrix T(k): L_b = sum_a T(k)_ba H_(pi(a) xor pi(b))[a],
    H_s[a] = sum_m (-1)^|m and s| M_m[a] (m: the axes member m negates, pi:
    exponent parities) - the decomposition of the GPU's sign-class M2L, here
    with 3, 2 and 1 non-zero axes."""
    p, eps = 5, 0.4
    e = oracle.exponents(p)
    nc = len(e)
    par = (e[:, 0] & 1) << 2 | (e[:, 1] & 1) << 1 | (e[:, 2] & 1)
    k = np.array(rep, dtype=float)
    zero = sum(4 >> d for d in range(3) if rep[d] == 0)
    members = [m for m in range(8) if not (m & zero)]
    rng = np.random.default_rng(5)
    Ms = {m: rng.normal(size=nc) / (1.0 + e.sum(axis=1)) for m in members}
    tgt = np.zeros(3)
    lhs = np.zeros(nc)
    for m in members:
        s = np.array([-1.0 if (m >> (2 - d)) & 1 else 1.0 for d in range(3)])
        lhs += oracle.soft_m2l(p, eps, tgt - s * k, tgt, Ms[m])
    # the representative's matrix, column by column
    T = np.stack([oracle.soft_m2l(p, eps, tgt - k, tgt, np.eye(nc)[a]) for a in range(nc)], axis=1)
    H = np.zeros((8, nc))
    for sgm in range(8):
        for m in members:
            H[sgm] += (-1.0) ** bin(m & sgm).count("1") * Ms[m]
    rhs = np.array([sum(T[b, a] * H[par[a] ^ par[b], a] for a in range(nc)) for b in range(nc)])
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(lhs))
