"""GPU FMM for the softened Coulomb kernel 1/sqrt(r^2 + eps^2) (the second
non-oscillatory kernel) against the oracle's softened DA-FMM.

Potentials and fields equal the oracle to relative L2 1e-12 on uniform trees
of depth 0-4 and on adaptive trees with W and X lists, orders 0-10, eps from 0
to well above the leaf size, ragged and clustered point sets and coincident
points; the multipole moments and local
Taylor coefficients match coefficient by coefficient; eps = 0 reproduces the
Coulomb path; at 1e6 points the potentials are checked against the softened
direct sum on sampled targets."""
import numpy as np
import pytest

import oracle
from paper_2508_02626_amd import fmm, inputs
from gpu_util import gpu_solve, oracle_tree, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


def soft_kw(depth, eps):
    return dict(uniform_depth=depth, root=[0, 0, 0, 1], kernel="softened", softening=eps)


def _check(x, q, p, depth, eps, tol=1e-12):
    kw = soft_kw(depth, eps)
    pl, phi, fld = gpu_solve(x, q, p, **kw)
    t = oracle_tree(x, **kw)
    ophi, ofld = t.fmm_soft(p, q, eps)
    e_phi, e_fld = rel_l2(phi, ophi), rel_l2(fld, ofld)
    say("  softened p=%d depth=%d eps=%g rel L2 vs oracle: phi %.3e field %.3e" % (p, depth, eps, e_phi, e_fld))
    assert e_phi <= tol and e_fld <= tol
    pl.close()
    return phi, fld


def _coincident(n, seed):
    x, q = inputs.uniform(n, seed)
    x[5] = x[1]
    x[n - 1] = x[1]
    return x, q


def _gauss_in_cube(n, seed):
    x, q = inputs.gaussian(n, seed, sigma=0.12)
    return np.clip(x + 0.5, 0.0, 1.0 - 1e-12), q


CASES = [
    ("uniform2000_p0", lambda: inputs.uniform(2000, 0), 0, 3, 0.01),
    ("uniform2000_p1", lambda: inputs.uniform(2000, 0), 1, 3, 0.01),
    ("uniform2000_p2", lambda: inputs.uniform(2000, 0), 2, 3, 0.01),
    ("uniform2000_p4", lambda: inputs.uniform(2000, 0), 4, 3, 0.01),
    ("uniform2000_p6_eps0", lambda: inputs.uniform(2000, 0), 6, 3, 0.0),
    ("uniform2000_p8", lambda: inputs.uniform(2000, 0), 8, 3, 0.01),
    ("uniform2000_p9_eps02", lambda: inputs.uniform(2000, 1), 9, 3, 0.2),
    ("uniform2000_p10", lambda: inputs.uniform(2000, 2), 10, 3, 0.003),
    ("uniform1_depth0", lambda: inputs.uniform(1, 3), 4, 0, 0.01),
    ("uniform37_depth1", lambda: inputs.uniform(37, 4), 5, 1, 0.05),
    ("uniform500_depth2", lambda: inputs.uniform(500, 5), 7, 2, 0.02),
    ("coincident_eps", lambda: _coincident(700, 6), 5, 2, 0.05),
    ("coincident_eps0", lambda: _coincident(700, 6), 5, 2, 0.0),
    ("gauss6000_depth4", lambda: _gauss_in_cube(6000, 7), 6, 4, 0.004),
]


@pytest.mark.parametrize("name,gen,p,depth,eps", CASES, ids=[c[0] for c in CASES])
def test_softened_matches_oracle(name, gen, p, depth, eps):
    x, q = gen()
    say("softened", name)
    _check(x, q, p, depth, eps)


def soft_kw_adaptive(s, eps):
    return dict(leaf_size=s, kernel="softened", softening=eps)


ADAPTIVE = [
    ("clusters_4000_s16_p5", lambda: inputs.clusters(4000, 3), 5, 16, 0.01),
    ("plummer_6000_s32_p7", lambda: inputs.plummer(6000, 2), 7, 32, 0.003),
    ("plummer_6000_s32_p2_eps0", lambda: inputs.plummer(6000, 2), 2, 32, 0.0),
    ("gaussian_5000_s50_p8", lambda: inputs.gaussian(5000, 4), 8, 50, 0.05),
    ("clusters_3000_s8_p10", lambda: inputs.clusters(3000, 9), 10, 8, 0.002),
    ("ragged_777_s5_p4", lambda: inputs.uniform(777, 5), 4, 5, 0.02),
]


@pytest.mark.parametrize("name,gen,p,leaf,eps", ADAPTIVE, ids=[c[0] for c in ADAPTIVE])
def test_softened_adaptive_matches_oracle(name, gen, p, leaf, eps):
    """Adaptive trees: M2L over level-ordered target tiles, P2L (X lists) and
    M2P (W lists) from the kernel's Taylor coefficients at the particles."""
    x, q = gen()
    say("softened adaptive", name)
    kw = soft_kw_adaptive(leaf, eps)
    t = oracle_tree(x, **kw)
    assert t.nV > 0
    pl, phi, fld = gpu_solve(x, q, p, **kw)
    ophi, ofld = t.fmm_soft(p, q, eps)
    e_phi, e_fld = rel_l2(phi, ophi), rel_l2(fld, ofld)
    say("  W %d X %d: rel L2 vs oracle phi %.3e field %.3e" % (t.nW, t.nX, e_phi, e_fld))
    assert e_phi <= 1e-12 and e_fld <= 1e-12
    pl.close()


def test_softened_adaptive_has_w_and_x_lists():
    """The adaptive cases above exercise P2L and M2P (non-empty X and W lists)."""
    x, q = inputs.clusters(4000, 3)
    t = oracle_tree(x, leaf_size=16)
    assert t.nW > 0 and t.nX > 0


def test_softened_adaptive_expansions_and_eps0():
    """Adaptive tree: M and L coefficient by coefficient; at eps = 0 the
    softened pipeline equals the Coulomb pipeline."""
    x, q = inputs.plummer(8000, 21)
    p, eps = 6, 0.004
    kw = soft_kw_adaptive(24, eps)
    pl, phi, fld = gpu_solve(x, q, p, **kw)
    M, L = pl.export_expansions()
    t = oracle_tree(x, **kw)
    assert t.nW > 0 and t.nX > 0
    _, _, oM, oL = t.fmm_soft(p, q, eps, want_expansions=True)
    deg = oracle.exponents(p).sum(axis=1)
    for d in range(p + 1):
        sel = deg == d
        assert np.abs(M[:, sel] - oM[:, sel]).max() <= 1e-12 * np.abs(oM[:, sel]).max(), ("M", d)
        assert np.abs(L[:, sel] - oL[:, sel]).max() <= 1e-12 * np.abs(oL[:, sel]).max(), ("L", d)
    pl.close()
    _, a, fa = gpu_solve(x, q, p, **soft_kw_adaptive(24, 0.0))
    _, b, fb = gpu_solve(x, q, p, leaf_size=24)
    say("  adaptive eps=0 vs Coulomb path: phi %.3e field %.3e" % (rel_l2(a, b), rel_l2(fa, fb)))
    assert rel_l2(a, b) <= 1e-12 and rel_l2(fa, fb) <= 1e-12


@pytest.mark.parametrize("p", [3, 8])
def test_softened_expansions_match_oracle(p):
    """Moments and local Taylor coefficients, degree by degree."""
    x, q = inputs.uniform(3000, 9)
    eps = 0.015
    kw = soft_kw(3, eps)
    pl, phi, fld = gpu_solve(x, q, p, **kw)
    M, L = pl.export_expansions()
    _, _, oM, oL = oracle_tree(x, **kw).fmm_soft(p, q, eps, want_expansions=True)
    deg = oracle.exponents(p).sum(axis=1)
    for d in range(p + 1):
        s = deg == d
        sm, sl = np.abs(oM[:, s]).max(), np.abs(oL[:, s]).max()
        assert np.abs(M[:, s] - oM[:, s]).max() <= 1e-12 * sm + 1e-300, ("M", d)
        assert np.abs(L[:, s] - oL[:, s]).max() <= 1e-12 * sl + 1e-300, ("L", d)
    pl.close()


def test_softened_eps0_equals_coulomb_path():
    """At eps = 0 the softened pipeline (full expansions, per-level tables)
    and the Coulomb pipeline (folded harmonic expansions, sign classes) compute
    the same truncated FMM."""
    x, q = inputs.uniform(5000, 10)
    _, a, fa = gpu_solve(x, q, 8, **soft_kw(4, 0.0))
    _, b, fb = gpu_solve(x, q, 8, uniform_depth=4, root=[0, 0, 0, 1])
    say("  eps=0 vs Coulomb path: phi %.3e field %.3e" % (rel_l2(a, b), rel_l2(fa, fb)))
    assert rel_l2(a, b) <= 1e-12 and rel_l2(fa, fb) <= 1e-12


def test_softened_mid_size_matches_oracle():
    """2e5 points, depth 4, p = 8: the launch shapes of the larger workload
    (interior tiles with all 189 offsets, several levels of tables)."""
    x, q = inputs.uniform(200_000, 11)
    _check(x, q, 8, 4, 1e-3)


def test_softened_full_size_sampled_direct():
    """1e6 uniform points, depth 5, p = 8, eps = 1e-3: the error against the
    softened direct sum on 2000 sampled targets is the truncation error."""
    x, q = inputs.uniform(1_000_000, 1)
    eps = 1e-3
    pl, phi, fld = gpu_solve(x, q, 8, **soft_kw(5, eps))
    idx = np.random.default_rng(12).choice(len(q), 2000, replace=False)
    d, fd = oracle.direct_soft(x, q, eps, targets=idx)
    e = rel_l2(phi[idx], d)
    say("  1e6 softened p=8 sigma vs direct (sampled): %.3e" % e)
    assert e < 5e-5
    pl.close()


def test_softened_deterministic_and_batch_refused():
    x, q = inputs.uniform(20_000, 13)
    pl = fmm.Plan(to_dev(x), 6, **soft_kw(3, 0.01))
    qt = to_dev(q)
    a, fa = pl.evaluate(qt)
    b, fb = pl.evaluate(qt)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()) and np.array_equal(fa.cpu().numpy(), fb.cpu().numpy())
    with pytest.raises(fmm.FmmError):
        fmm.evaluate_batch([pl], [qt])
    pl.close()


def test_softened_plummer_full_size_sampled_direct():
    """The softened_plummer1m benchmark shape: 1e6 Plummer points (seed 2),
    adaptive s = 64, p = 8, eps = 1e-4 (W and X lists at every level, M2L
    tiles spanning two levels, two blocks per tile adding into L).  The
    potentials against the softened direct sum on 2000 sampled targets carry
    the truncation error only; two evaluations agree bit for bit."""
    x, q = inputs.plummer(1_000_000, 2)
    eps = 1e-4
    kw = soft_kw_adaptive(64, eps)
    pl = fmm.Plan(to_dev(x), 8, **kw)
    qt = to_dev(q)
    a, fa = pl.evaluate(qt)
    b, fb = pl.evaluate(qt)
    a, fa, b, fb = a.cpu().numpy(), fa.cpu().numpy(), b.cpu().numpy(), fb.cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    idx = np.random.default_rng(14).choice(len(q), 2000, replace=False)
    d, fd = oracle.direct_soft(x, q, eps, targets=idx)
    e, ef = rel_l2(a[idx], d), rel_l2(fa[idx], fd)
    say("  1e6 Plummer softened p=8 sigma vs direct (sampled): phi %.3e field %.3e" % (e, ef))
    assert e < 5e-5 and ef < 5e-4
    pl.close()
