"""Parity at the sizes of the benchmark configurations.

* 1e6 uniform points, depth 5, p = 8 (the uniform benchmark workload, in the
  launch configuration the benchmark times): the whole FP64 result against the
  oracle DA-FMM at 1e-12 relative L2 (potential and field); each FP32 part of
  the mixed path, alone and together, with its error against the oracle stated
  and bounded.
* An adaptive Plummer tree (3e4 points, s = 64: W and X lists, full V lists)
  at p = 10 and p = 14 in FP64 against the oracle at 1e-12, with the
  multipole and local expansions compared coefficient by coefficient at
  p = 10 (the parents' multipoles are the evaluation's own folded M2M output).
* 4e6 Plummer points at p = 14 (the metric's workload): sampled relative
  error against the direct sum at most 1e-7, FP64 and mixed.
"""
import numpy as np
import pytest

import oracle
from paper_2508_02626_amd import inputs
from gpu_util import gpu_solve, oracle_tree, rel_l2, say

pytestmark = pytest.mark.gpu

UNI = dict(uniform_depth=5, root=[0, 0, 0, 1])
_cache = {}


def _oracle_fmm(key, x, q, p, kw, expansions=False):
    if key not in _cache:
        say("  oracle DA-FMM", key)
        _cache[key] = oracle_tree(x, **kw).fmm(p, q, want_expansions=expansions)
    return _cache[key]


def test_uniform1m_fp64_whole_result_matches_oracle():
    x, q = inputs.uniform(1_000_000, 1)
    ophi, ofld = _oracle_fmm("uniform1m", x, q, 8, UNI)
    pl, phi, fld = gpu_solve(x, q, 8, **UNI)
    pl.close()
    e_phi, e_fld = rel_l2(phi, ophi), rel_l2(fld, ofld)
    say("  uniform1m p=8 FP64 rel L2 vs oracle: phi %.3e field %.3e" % (e_phi, e_fld))
    assert e_phi <= 1e-12 and e_fld <= 1e-12


# stated bounds of each FP32 part against the FP64 oracle (relative L2 of the
# potential, of the field)
@pytest.mark.parametrize("prec,bound,bound_f", [("p2p32", 5e-8, 3e-7), ("m2l32", 3e-7, 1e-6),
                                                ("mixed", 3e-7, 1e-6)])
def test_uniform1m_mixed_parts_error_against_oracle(prec, bound, bound_f):
    x, q = inputs.uniform(1_000_000, 1)
    ophi, ofld = _oracle_fmm("uniform1m", x, q, 8, UNI)
    pl, phi, fld = gpu_solve(x, q, 8, precision=prec, **UNI)
    pl.close()
    e_phi, e_fld = rel_l2(phi, ophi), rel_l2(fld, ofld)
    say("  uniform1m p=8 %s rel L2 vs oracle: phi %.3e field %.3e" % (prec, e_phi, e_fld))
    assert e_phi <= bound and e_fld <= bound_f


@pytest.mark.parametrize("p", [10, 14])
def test_adaptive_plummer_matches_oracle(p):
    x, q = inputs.plummer(30_000, 11)
    kw = dict(leaf_size=64)
    want = p == 10
    res = _oracle_fmm(("plummer3e4", p), x, q, p, kw, expansions=want)
    ophi, ofld = res[0], res[1]
    pl, phi, fld = gpu_solve(x, q, p, **kw)
    s = pl.sizes()
    say("  plummer 3e4 s=64 sizes", s)
    assert s["W"] > 10_000 and s["X"] > 10_000 and s["V"] > 100_000
    e_phi, e_fld = rel_l2(phi, ophi), rel_l2(fld, ofld)
    say("  plummer 3e4 p=%d FP64 rel L2 vs oracle: phi %.3e field %.3e" % (p, e_phi, e_fld))
    assert e_phi <= 1e-12 and e_fld <= 1e-12
    if want:
        oM, oL = res[2], res[3]
        M, L = pl.export_expansions()
        deg = oracle.exponents(p).sum(axis=1)
        for d in range(p + 1):
            sel = deg == d
            sm, sl = np.abs(oM[:, sel]).max(), np.abs(oL[:, sel]).max()
            assert np.abs(M[:, sel] - oM[:, sel]).max() <= 1e-12 * sm, ("M", d)
            assert np.abs(L[:, sel] - oL[:, sel]).max() <= 1e-12 * sl, ("L", d)
    pl.close()


@pytest.mark.parametrize("p", [10, 14])
def test_adaptive_plummer_rotation_m2l_matches_oracle(p):
    """The rotation-based M2L (Sec. 3.4) on the Plummer tree with full V
    lists: FP64 potentials and fields equal the oracle to 1e-12."""
    x, q = inputs.plummer(30_000, 11)
    kw = dict(leaf_size=64)
    res = _oracle_fmm(("plummer3e4", p), x, q, p, kw, expansions=p == 10)
    pl, phi, fld = gpu_solve(x, q, p, m2l="rotation", **kw)
    pl.close()
    e_phi, e_fld = rel_l2(phi, res[0]), rel_l2(fld, res[1])
    say("  plummer 3e4 p=%d rotation M2L rel L2 vs oracle: phi %.3e field %.3e" % (p, e_phi, e_fld))
    assert e_phi <= 1e-12 and e_fld <= 1e-12


@pytest.mark.parametrize("p", [12, 14])
def test_adaptive_plummer_mixed_error_against_oracle(p):
    """Mixed path at orders >= 12: FP32 P2P terms with compensated sums and
    FP32 MFMA for the M2L row tiles after the first row part (the higher
    degrees); stated error against the FP64 oracle."""
    x, q = inputs.plummer(30_000, 11)
    kw = dict(leaf_size=64)
    res = _oracle_fmm(("plummer3e4", p), x, q, p, kw, expansions=p == 10)
    pl, phi, fld = gpu_solve(x, q, p, precision="mixed", **kw)
    pl.close()
    e_phi, e_fld = rel_l2(phi, res[0]), rel_l2(fld, res[1])
    say("  plummer 3e4 p=%d mixed rel L2 vs oracle: phi %.3e field %.3e" % (p, e_phi, e_fld))
    assert e_phi <= 1e-7 and e_fld <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plummer4m_meets_1e7_at_order_14(prec):
    x, q = inputs.plummer(4_000_000, 2)
    idx = np.sort(np.random.default_rng(7).choice(len(q), 1000, replace=False))
    if "direct4m" not in _cache:
        _cache["direct4m"] = oracle.direct(x, q, idx)
    d, fd = _cache["direct4m"]
    pl, phi, fld = gpu_solve(x, q, 14, leaf_size=64, precision=prec)
    pl.close()
    e, ef = rel_l2(phi[idx], d), rel_l2(fld[idx], fd)
    say("  plummer 4e6 p=14 %s sampled sigma phi %.3e field %.3e" % (prec, e, ef))
    assert e <= 1e-7 and ef <= 1e-6
