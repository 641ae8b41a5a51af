"""CPU oracle for the DA-FMM (arXiv 2508.02626): ctypes binding of liboracle.so.

TEST INFRASTRUCTURE ONLY.  The oracle is the plain FP64 reference the GPU path
is checked against.  Only tests, the smoke check and the benchmark's CPU
baseline may import it; the product package never does, and the two share no
code.  See oracle.h for what each C function follows in the paper.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = ["tpsa.c", "direct.c", "tree.c", "dafmm.c", "soft.c"]


def build(verbose=False):
    """Compile liboracle.so with gcc (plain C99 + OpenMP, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-D_POSIX_C_SOURCE=200809L", "-o", _SO + ".tmp"] + [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        dp = P(d)
        L.oracle_da_inv_r.argtypes = [i32, dp, dp]
        L.oracle_da_op.argtypes = [i32, i32, dp, dp, dp]
        L.oracle_da_compose.argtypes = [i32, dp, i32, dp, dp]
        L.oracle_p2m.argtypes = [i32, i64, dp, dp, dp, dp]
        L.oracle_p2l.argtypes = [i32, i64, dp, dp, dp, dp]
        L.oracle_m2m.argtypes = [i32, dp, dp, dp, dp]
        L.oracle_m2l.argtypes = [i32, dp, dp, dp, dp]
        L.oracle_l2l.argtypes = [i32, dp, dp, dp, dp]
        L.oracle_l2p.argtypes = [i32, dp, dp, i64, dp, dp, dp]
        L.oracle_m2p.argtypes = [i32, dp, dp, i64, dp, dp, dp]
        L.oracle_direct.argtypes = [i64, dp, dp, i64, P(i64), dp, dp]
        L.oracle_tree_build.restype = ctypes.c_void_p
        L.oracle_tree_build.argtypes = [i64, dp, dp, i32, i32, i32]
        L.oracle_tree_free.argtypes = [ctypes.c_void_p]
        L.oracle_tree_sizes.argtypes = [ctypes.c_void_p, P(i64)]
        L.oracle_tree_root.argtypes = [ctypes.c_void_p, dp]
        L.oracle_tree_export.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 16
        L.oracle_fmm.argtypes = [ctypes.c_void_p, i32, dp, dp, i32, dp, dp, dp, dp]
        L.oracle_soft_taylor.argtypes = [i32, dp, d, dp]
        L.oracle_direct_soft.argtypes = [i64, dp, dp, d, i64, P(i64), dp, dp]
        L.oracle_soft_op.argtypes = [i32, i32, d, dp, dp, dp, dp]
        L.oracle_soft_p2m.argtypes = [i32, i64, dp, dp, dp, dp]
        L.oracle_soft_p2l.argtypes = [i32, d, i64, dp, dp, dp, dp]
        L.oracle_fmm_soft.argtypes = [ctypes.c_void_p, i32, d, dp, dp, dp, dp, dp, dp]
        L.oracle_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def ncoef(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def exponents(p):
    """Monomial exponents in the oracle's DA order (Table 1 order)."""
    out = []
    for n in range(p + 1):
        for i in range(n, -1, -1):
            for j in range(n - i, -1, -1):
                out.append((i, j, n - i - j))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def num_threads():
    return lib().oracle_num_threads()


def da_inv_r(p, x0):
    out = np.zeros(ncoef(p))
    x0 = _c(x0)
    assert lib().oracle_da_inv_r(p, _p(x0), _p(out)) == 0
    return out


def da_op(op, p, a, b=None):
    """op: 'mul', 'inv', 'sqrt', 'dx', 'dy', 'dz' on DA vectors of order p."""
    code = {"mul": 0, "inv": 1, "sqrt": 2, "dx": 3, "dy": 4, "dz": 5}[op]
    a = _c(a)
    b = a if b is None else _c(b)
    out = np.zeros(ncoef(p))
    assert lib().oracle_da_op(code, p, _p(a), _p(b), _p(out)) == 0
    return out


def da_compose(p, f, q, args):
    """f (order p) o (args[0], args[1], args[2]) (order-q DA vectors)."""
    f, args = _c(f), _c(args)
    out = np.zeros(ncoef(q))
    assert lib().oracle_da_compose(p, _p(f), q, _p(args), _p(out)) == 0
    return out


def p2m(p, xyz, q, center):
    xyz, q, center = _c(xyz), _c(q), _c(center)
    M = np.zeros(ncoef(p))
    assert lib().oracle_p2m(p, len(q), _p(xyz), _p(q), _p(center), _p(M)) == 0
    return M


def p2l(p, xyz, q, center):
    xyz, q, center = _c(xyz), _c(q), _c(center)
    L = np.zeros(ncoef(p))
    assert lib().oracle_p2l(p, len(q), _p(xyz), _p(q), _p(center), _p(L)) == 0
    return L


def _translate(fn, p, a, b, v):
    a, b, v = _c(a), _c(b), _c(v)
    out = np.zeros(ncoef(p))
    assert fn(p, _p(a), _p(b), _p(v), _p(out)) == 0
    return out


def m2m(p, child_center, parent_center, M):
    return _translate(lib().oracle_m2m, p, child_center, parent_center, M)


def m2l(p, src_center, tgt_center, M):
    return _translate(lib().oracle_m2l, p, src_center, tgt_center, M)


def l2l(p, parent_center, child_center, L):
    return _translate(lib().oracle_l2l, p, parent_center, child_center, L)


def _eval(fn, p, center, v, xyz):
    center, v, xyz = _c(center), _c(v), _c(np.atleast_2d(xyz))
    phi = np.zeros(len(xyz))
    field = np.zeros((len(xyz), 3))
    assert fn(p, _p(center), _p(v), len(xyz), _p(xyz), _p(phi), _p(field)) == 0
    return phi, field


def l2p(p, center, L, xyz):
    return _eval(lib().oracle_l2p, p, center, L, xyz)


def m2p(p, center, M, xyz):
    return _eval(lib().oracle_m2p, p, center, M, xyz)


def direct(xyz, q, targets=None):
    """Direct sum: (phi, field) at the targets (all particles if None)."""
    xyz, q = _c(xyz), _c(q)
    n = len(q)
    if targets is None:
        nt, tp = n, None
    else:
        targets = _c(targets, np.int64)
        nt, tp = len(targets), targets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    phi = np.zeros(nt)
    field = np.zeros((nt, 3))
    assert lib().oracle_direct(n, _p(xyz), _p(q), nt, tp, _p(phi), _p(field)) == 0
    return phi, field


# ---- softened Coulomb kernel K(x) = 1/sqrt(|x|^2 + eps^2) (soft.c) ----
def soft_taylor(p, x0, eps):
    """Taylor coefficients of K(x0 + z) in z (DA order), by the DA algebra."""
    out = np.zeros(ncoef(p))
    x0 = _c(x0)
    assert lib().oracle_soft_taylor(p, _p(x0), float(eps), _p(out)) == 0
    return out


def direct_soft(xyz, q, eps, targets=None):
    xyz, q = _c(xyz), _c(q)
    n = len(q)
    if targets is None:
        nt, tp = n, None
    else:
        targets = _c(targets, np.int64)
        nt, tp = len(targets), targets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    phi = np.zeros(nt)
    field = np.zeros((nt, 3))
    assert lib().oracle_direct_soft(n, _p(xyz), _p(q), float(eps), nt, tp, _p(phi), _p(field)) == 0
    return phi, field


def _soft_op(op, p, eps, a3, b3, v):
    a3, b3, v = _c(a3), _c(b3), _c(v)
    out = np.zeros(ncoef(p))
    assert lib().oracle_soft_op(op, p, float(eps), _p(a3), _p(b3), _p(v), _p(out)) == 0
    return out


def soft_m2m(p, child_center, parent_center, M):
    return _soft_op(0, p, 0.0, child_center, parent_center, M)


def soft_m2l(p, eps, src_center, tgt_center, M):
    return _soft_op(1, p, eps, src_center, tgt_center, M)


def soft_l2l(p, parent_center, child_center, L):
    return _soft_op(2, p, 0.0, parent_center, child_center, L)


def soft_p2m(p, xyz, q, center):
    xyz, q, center = _c(xyz), _c(q), _c(center)
    M = np.zeros(ncoef(p))
    assert lib().oracle_soft_p2m(p, len(q), _p(xyz), _p(q), _p(center), _p(M)) == 0
    return M


def soft_p2l(p, eps, xyz, q, center):
    xyz, q, center = _c(xyz), _c(q), _c(center)
    L = np.zeros(ncoef(p))
    assert lib().oracle_soft_p2l(p, float(eps), len(q), _p(xyz), _p(q), _p(center), _p(L)) == 0
    return L


class Tree:
    """Reference octree + CGR interaction lists (tree.c)."""

    def __init__(self, xyz, root=None, uniform_depth=-1, max_depth=21, leaf_size=64):
        self.xyz = _c(xyz)
        r = None if root is None else _c(root)
        h = lib().oracle_tree_build(len(self.xyz), _p(self.xyz), None if r is None else _p(r),
                                    uniform_depth, max_depth, leaf_size)
        if not h:
            raise ValueError("oracle_tree_build rejected its arguments")
        self._h = ctypes.c_void_p(h)
        s = np.zeros(7, dtype=np.int64)
        lib().oracle_tree_sizes(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        self.nboxes, self.nU, self.nV, self.nW, self.nX, self.depth, self.key_depth = map(int, s)
        rt = np.zeros(4)
        lib().oracle_tree_root(self._h, _p(rt))
        self.root = rt

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_tree_free(h)
            self._h = None

    def export(self):
        nb = self.nboxes
        d = dict(perm=np.zeros(len(self.xyz), np.int64), level=np.zeros(nb, np.int32),
                 morton=np.zeros(nb, np.uint64), first=np.zeros(nb, np.int64),
                 count=np.zeros(nb, np.int64), parent=np.zeros(nb, np.int32),
                 child_begin=np.zeros(nb, np.int32), nchild=np.zeros(nb, np.int32))
        for k, m in (("U", self.nU), ("V", self.nV), ("W", self.nW), ("X", self.nX)):
            d[k + "_off"] = np.zeros(nb + 1, np.int64)
            d[k + "_src"] = np.zeros(max(m, 1), np.int32)
        keys = ["perm", "level", "morton", "first", "count", "parent", "child_begin", "nchild",
                "U_off", "U_src", "V_off", "V_src", "W_off", "W_src", "X_off", "X_src"]
        lib().oracle_tree_export(self._h, *[ctypes.c_void_p(d[k].ctypes.data) for k in keys])
        for k, m in (("U", self.nU), ("V", self.nV), ("W", self.nW), ("X", self.nX)):
            d[k + "_src"] = d[k + "_src"][:m]
        return d

    def fmm(self, p, q, memo=True, want_expansions=False):
        """DA-FMM potentials and fields (original particle order)."""
        q = _c(q)
        n = len(q)
        phi = np.zeros(n)
        field = np.zeros((n, 3))
        M = L = None
        if want_expansions:
            M = np.zeros((self.nboxes, ncoef(p)))
            L = np.zeros((self.nboxes, ncoef(p)))
        rc = lib().oracle_fmm(self._h, p, _p(self.xyz), _p(q), 1 if memo else 0, _p(phi), _p(field),
                              None if M is None else _p(M), None if L is None else _p(L))
        assert rc == 0
        if want_expansions:
            return phi, field, M, L
        return phi, field

    def fmm_soft(self, p, q, eps, want_expansions=False):
        """Softened-kernel FMM (soft.c): potentials and fields; M and L (box
        order, physical units: moments and local Taylor coefficients)."""
        q = _c(q)
        n = len(q)
        phi = np.zeros(n)
        field = np.zeros((n, 3))
        M = L = None
        if want_expansions:
            M = np.zeros((self.nboxes, ncoef(p)))
            L = np.zeros((self.nboxes, ncoef(p)))
        rc = lib().oracle_fmm_soft(self._h, p, float(eps), _p(self.xyz), _p(q), _p(phi), _p(field),
                                   None if M is None else _p(M), None if L is None else _p(L))
        assert rc == 0
        if want_expansions:
            return phi, field, M, L
        return phi, field
