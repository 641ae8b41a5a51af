"""The library's per-order constant tables (fmm_order_table, built on the host
from closed forms) against what the paper and the oracle fix, on the CPU:

* derivative tables: d^g (1/|x|) at integer offsets equal g! times the
  oracle's Taylor coefficients of 1/|x0 + d| (pinned to Table 1), and a few
  entries equal exact sympy derivatives;
* M2M octant matrices: translating the P2M multipole of a child box equals
  the oracle's DA M2M (Eq. m2m) of the same multipole;
* L2L octant matrices: equal the oracle's DA L2L (Eq. l2l) on any polynomial;
* P2M map: raw moments times the map equal the oracle's P2M (Eq. P2M);
* harmonic reconstruction: the full multipole is recovered exactly from its
  components with z exponent <= 1, the fold being written out here from
  Laplace's equation (d_z^2 = -(d_x^2 + d_y^2) on 1/r);
* folded multipole layout: every component is kept exactly once, and at the
  sign-class orders the columns read back in k-step order run through the
  parity classes in order, each padded to whole k-steps of four.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2508_02626_amd import fmm


def exps(p):
    return oracle.exponents(p)


def w(n):
    df = 1.0
    for t in range(2 * n - 1, 1, -2):
        df *= t
    return (-1) ** n / df


def per_degree_close(a, b, p, tol):
    deg = exps(p).sum(axis=1)
    for d in range(p + 1):
        s = deg == d
        scale = max(np.abs(b[..., s]).max(), 1e-300)
        assert np.abs(a[..., s] - b[..., s]).max() <= tol * scale, d


def compact_index(p):
    """(i, j, z) of each entry of a derivative-table row."""
    out = []
    for z in range(3):
        for i in range(2 * p + 1 - z):
            for j in range(2 * p + 1 - z - i):
                out.append((i, j, z))
    return out


@pytest.mark.parametrize("p", [3, 6])
def test_derivative_tables_equal_oracle_taylor_coefficients(p):
    D = fmm.order_table(p, 0)
    ent = compact_index(p)
    E = exps(2 * p)
    pos = {tuple(e): k for k, e in enumerate(E)}
    checked = 0
    for kx in range(-3, 4):
        for ky in range(-3, 4):
            for kz in range(-3, 4):
                row = D[(kx + 3) * 49 + (ky + 3) * 7 + (kz + 3)]
                if max(abs(kx), abs(ky), abs(kz)) <= 1:
                    assert not row.any()
                    continue
                a = oracle.da_inv_r(2 * p, [kx, ky, kz])
                ref = np.array([a[pos[e]] * math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2])
                                for e in ent])
                got = row[:len(ent)]
                deg = np.array([sum(e) for e in ent])
                for d in range(2 * p + 1):
                    s = deg == d
                    assert np.abs(got[s] - ref[s]).max() <= 1e-13 * np.abs(ref[s]).max(), (kx, ky, kz, d)
                checked += 1
    assert checked == 316


def test_derivative_table_entries_equal_sympy():
    sympy = pytest.importorskip("sympy")
    p = 4
    D = fmm.order_table(p, 0)
    ent = compact_index(p)
    X, Y, Z = sympy.symbols("x y z")
    f = 1 / sympy.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    for k in [(2, 1, 0), (-3, 2, 1), (3, -3, -2), (0, 0, 2)]:
        row = D[(k[0] + 3) * 49 + (k[1] + 3) * 7 + (k[2] + 3)]
        for e in [(0, 0, 0), (1, 0, 0), (2, 1, 1), (5, 0, 2), (3, 3, 2), (0, 7, 1)]:
            exact = sympy.diff(f, X, e[0], Y, e[1], Z, e[2]).subs({X: k[0], Y: k[1], Z: k[2]})
            v = float(sympy.N(exact, 30))
            assert abs(row[ent.index(e)] - v) <= 1e-14 * max(abs(v), 1e-300), (k, e)


def box_particles(rng, centre, h, m=40):
    return centre + (rng.random((m, 3)) - 0.5) * h, rng.uniform(-1, 1, m)


@pytest.mark.parametrize("p", [4, 7])
def test_m2m_tables_equal_oracle_m2m(p):
    S = fmm.order_table(p, 1)
    nc = oracle.ncoef(p)
    S = S.reshape(8, nc, nc)
    deg = exps(p).sum(axis=1)
    wd = np.array([w(d) for d in deg])
    rng = np.random.default_rng(3)
    h = 0.25
    for o in range(8):
        tau = np.array([0.5 if (o >> (2 - k)) & 1 else -0.5 for k in range(3)])
        child = np.array([0.3, -0.2, 0.7])
        parent = child - tau * h
        x, q = box_particles(rng, child, h)
        M = oracle.p2m(p, x, q, child)
        Mh = wd * M / h ** deg
        pred = Mh @ S[o]
        ref = oracle.m2m(p, child, parent, M)
        refh = wd * ref / (2 * h) ** deg
        per_degree_close(pred, refh, p, 1e-13)
        # and the translation is exact: it equals P2M about the parent
        direct = wd * oracle.p2m(p, x, q, parent) / (2 * h) ** deg
        per_degree_close(pred, direct, p, 1e-12)


@pytest.mark.parametrize("p", [4, 7])
def test_l2l_tables_equal_oracle_l2l(p):
    G = fmm.order_table(p, 2)
    nc = oracle.ncoef(p)
    G = G.reshape(8, nc, nc)
    E = exps(p)
    deg = E.sum(axis=1)
    fac = np.array([math.factorial(a) * math.factorial(b) * math.factorial(c) for a, b, c in E], float)
    rng = np.random.default_rng(4)
    h = 0.125
    H = 2 * h
    for o in range(8):
        tau = np.array([0.5 if (o >> (2 - k)) & 1 else -0.5 for k in range(3)])
        parent = np.array([-0.4, 0.1, 0.25])
        child = parent + tau * h
        L = rng.normal(size=nc)
        Lh = fac * L * H ** (deg + 1)
        pred = Lh @ G[o]
        ref = oracle.l2l(p, parent, child, L)
        refh = fac * ref * h ** (deg + 1)
        per_degree_close(pred, refh, p, 1e-13)


@pytest.mark.parametrize("p", [3, 8])
def test_p2m_map_equals_oracle_p2m(p):
    P = fmm.order_table(p, 3)
    E = exps(p)
    deg = E.sum(axis=1)
    wd = np.array([w(d) for d in deg])
    rng = np.random.default_rng(5)
    h, c = 0.5, np.array([0.1, 0.2, 0.3])
    x, q = box_particles(rng, c, h, 100)
    u = (x - c) / h
    Q = np.array([np.sum(q * u[:, 0] ** a * u[:, 1] ** b * u[:, 2] ** g) for a, b, g in E])
    pred = Q @ P
    ref = wd * oracle.p2m(p, x, q, c) / h ** deg
    per_degree_close(pred, ref, p, 1e-13)


def harmonic_components(p):
    out = []
    for n in range(p + 1):
        out += [(i, n - i, 0) for i in range(n, -1, -1)]
        out += [(i, n - 1 - i, 1) for i in range(n - 1, -1, -1)]
    return out


def fold(M, p):
    """Components (I, J, kz), kz <= 1, of a multipole whose far field
    sum_a M_a d^a(1/r) they reproduce: d^(i,j,k+2m)(1/r) =
    sum_a (-1)^m C(m,a) d^(i+2a, j+2(m-a), k)(1/r) (Laplace's equation)."""
    pos = {tuple(e): k for k, e in enumerate(exps(p))}
    out = []
    for I, J, kz in harmonic_components(p):
        s = 0.0
        m = 0
        while kz + 2 * m <= p:
            for a in range(m + 1):
                i, j = I - 2 * a, J - 2 * (m - a)
                if i >= 0 and j >= 0:
                    s += (-1) ** m * math.comb(m, a) * M[pos[(i, j, kz + 2 * m)]]
            m += 1
        out.append(s)
    return np.array(out)


@pytest.mark.parametrize("p", [5, 10])
def test_harmonic_reconstruction_inverts_the_fold(p):
    HR = fmm.order_table(p, 4)
    assert HR.shape == ((p + 1) ** 2, oracle.ncoef(p))
    rng = np.random.default_rng(6)
    c = np.array([0.0, 0.0, 0.0])
    x, q = box_particles(rng, c, 1.0, 60)
    M = oracle.p2m(p, x, q, c)
    rec = fold(M, p) @ HR
    per_degree_close(rec, M, p, 1e-12)


def test_order_table_rejects_bad_arguments():
    import ctypes
    cnt, ld = ctypes.c_int64(), ctypes.c_int32()
    L = fmm.lib()
    assert L.fmm_order_table(17, 0, None, 0, ctypes.byref(cnt), ctypes.byref(ld)) == fmm.FMM_EINVAL
    assert L.fmm_order_table(4, 10, None, 0, ctypes.byref(cnt), ctypes.byref(ld)) == fmm.FMM_EINVAL
    assert L.fmm_order_table(4, 1, None, 0, ctypes.byref(cnt), ctypes.byref(ld)) == fmm.FMM_OK
    buf = np.zeros(3)
    assert L.fmm_order_table(4, 1, ctypes.c_void_p(buf.ctypes.data), 3, ctypes.byref(cnt),
                             ctypes.byref(ld)) == fmm.FMM_EINVAL


def folded_components(n):
    return [(i, n - i, 0) for i in range(n, -1, -1)] + [(i, n - 1 - i, 1) for i in range(n - 1, -1, -1)]


def mode_index(m, t):
    return 0 if m == 0 else 2 * m - 1 + t


@pytest.mark.parametrize("p", [3, 8, 12])
def test_rotation_factors_reproduce_the_m2l_contraction(p):
    """Rotation-based M2L (Sec. 3.4): for each of the 316 offsets k, the rotated
    multipole map F, the axial map A (one block per azimuthal mode, the same
    for cos and sin) and the local map B give back the folded M2L matrix,
    T(k)[b][a] = d^(a+b)(1/|x|) at x = k, taken from the derivative tables:
    T(s o k) = R_s B A F R_s with the factors stored for |k|."""
    D = fmm.order_table(p, 0)
    F = fmm.order_table(p, 5)
    Bm = fmm.order_table(p, 6)
    A = fmm.order_table(p, 7)
    aidx = fmm.order_table(p, 8).ravel().astype(int)
    ent = {e: i for i, e in enumerate(compact_index(p))}
    offs = [0]
    for n in range(p + 1):
        offs.append(offs[-1] + (2 * n + 1) ** 2)
    aoff = [0]
    for m in range(p + 1):
        aoff.append(aoff[-1] + (p + 1 - m) ** 2)
    comps = [folded_components(n) for n in range(p + 1)]
    worst = 0.0
    for kx in range(-3, 4):
        for ky in range(-3, 4):
            for kz in range(-3, 4):
                if max(abs(kx), abs(ky), abs(kz)) <= 1:
                    continue
                row = D[(kx + 3) * 49 + (ky + 3) * 7 + (kz + 3)]
                cls = abs(kx) * 16 + abs(ky) * 4 + abs(kz)
                sg = (1 if kx >= 0 else -1, 1 if ky >= 0 else -1, 1 if kz >= 0 else -1)
                ar = A[aidx[cls]]
                for n in range(p + 1):
                    wn = 2 * n + 1
                    Fn = F[cls, offs[n]:offs[n + 1]].reshape(wn, wn).T  # [mode][a]
                    rn = np.array([sg[0] ** c[0] * sg[1] ** c[1] * sg[2] ** c[2] for c in comps[n]])
                    for l in range(p + 1):
                        wl = 2 * l + 1
                        Bl = Bm[cls, offs[l]:offs[l + 1]].reshape(wl, wl).T  # [b][mode]
                        rl = np.array([sg[0] ** c[0] * sg[1] ** c[1] * sg[2] ** c[2] for c in comps[l]])
                        Aln = np.zeros((wl, wn))
                        for m in range(min(l, n) + 1):
                            w = p + 1 - m
                            v = ar[aoff[m] + (n - m) * w + (l - m)]
                            for t in range(2 if m else 1):
                                Aln[mode_index(m, t), mode_index(m, t)] = v
                        pred = (rl[:, None] * (Bl @ Aln @ Fn)) * rn[None, :]
                        true = np.array([[row[ent[(b[0] + a[0], b[1] + a[1], b[2] + a[2])]] for a in comps[n]]
                                         for b in comps[l]])
                        err = np.abs(pred - true).max() / np.abs(true).max()
                        worst = max(worst, err)
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("p", [0, 3, 5, 6, 8, 11, 12, 13, 14, 16])
def test_folded_layout_keeps_each_component_once_in_class_order(p):
    """The folded-multipole row (table 9) against a layout derived here from
    the components' exponent parities: below order 6 the harmonic order; from
    6 on, read in k-step order (sorted column 4 s + g at 8 (s // 2) + 2 g +
    s % 2), the classes 4 (i % 2) + 2 (j % 2) + k come in increasing order,
    each class's components in harmonic order and padded with -1 to a
    multiple of 4, and the row length is 16 per four k-steps."""
    pos = fmm.order_table(p, 9)
    assert pos.shape[0] == 1
    pos = pos[0].astype(int)
    comps = harmonic_components(p)
    nh = (p + 1) ** 2
    assert len(comps) == nh
    kept = pos[pos >= 0]
    assert sorted(kept.tolist()) == list(range(nh))
    if p < 6:
        assert pos[:nh].tolist() == list(range(nh)) and (pos[nh:] == -1).all()
        assert len(pos) == (nh + 15) // 16 * 16
        return
    cls = [4 * (i % 2) + 2 * (j % 2) + k for i, j, k in comps]
    expect = []
    for c in range(8):
        members = [h for h in range(nh) if cls[h] == c]
        expect += members + [-1] * (-len(members) % 4)
    ks = len(expect) // 4
    assert len(pos) == 16 * ((ks + 3) // 4)
    sorted_cols = [pos[8 * (s // 2) + 2 * g + s % 2] for s in range(ks) for g in range(4)]
    assert sorted_cols == expect
    used = {8 * (s // 2) + 2 * g + s % 2 for s in range(ks) for g in range(4)}
    assert all(pos[q] == -1 for q in range(len(pos)) if q not in used)
