"""Python binding of libfmm_mi355x.so (include/fmm.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch tensors supply device memory and the current HIP stream.
There is no fallback: if the library is missing or no GPU is present the calls
raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm_mi355x.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_EUNSUPPORTED = 0, -1, -2, -3, -4
FMM_FP64, FMM_P2P_F32, FMM_M2L_F32, FMM_MIXED = 0, 1, 2, 3
PRECISIONS = {"fp64": FMM_FP64, "p2p32": FMM_P2P_F32, "m2l32": FMM_M2L_F32, "mixed": FMM_MIXED}

SYMBOLS = ["fmm_default_options", "fmm_plan", "fmm_evaluate", "fmm_evaluate_batch",
           "fmm_plan_footprint", "fmm_plan_estimate", "fmm_plan_sizes", "fmm_plan_export_tree",
           "fmm_plan_export_expansions", "fmm_plan_set_timing", "fmm_plan_read_timing",
           "fmm_plan_destroy", "fmm_last_error", "fmm_plan_batch", "fmm_cached_bytes",
           "fmm_order_table", "fmm_evaluate_batch_noalloc"]
STAGES = ["permute", "p2m", "m2m", "fold", "m2l", "p2l", "unfold", "l2l", "l2p", "p2p", "p2p_part2", "m2p"]


class FmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("uniform_depth", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("want_field", ctypes.c_int32),
                ("root", ctypes.POINTER(ctypes.c_double)), ("m2l_method", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("softening", ctypes.c_double)]


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p), ("ctx", ctypes.c_void_p)]


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FmmError(FMM_EUNSUPPORTED, "libfmm_mi355x.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER
        L.fmm_default_options.argtypes = [P(Options)]
        L.fmm_default_options.restype = None
        L.fmm_plan.argtypes = [vp, i64, i32, i32, P(Options), P(Allocator), vp, P(vp)]
        L.fmm_evaluate.argtypes = [vp, vp, vp, vp, vp]
        L.fmm_evaluate_batch.argtypes = [P(vp), P(vp), P(vp), P(vp), i32, vp]
        L.fmm_evaluate_batch_noalloc.argtypes = [P(vp), P(vp), P(vp), P(vp), i32, vp]
        L.fmm_plan_footprint.argtypes = [vp, P(ctypes.c_size_t)]
        L.fmm_plan_estimate.argtypes = [i64, i32, i32, P(Options), P(ctypes.c_size_t)]
        L.fmm_plan_sizes.argtypes = [vp, P(i64)]
        L.fmm_plan_export_tree.argtypes = [vp, vp] + [vp] * 17
        L.fmm_plan_export_expansions.argtypes = [vp, vp, vp, vp]
        L.fmm_plan_set_timing.argtypes = [vp, ctypes.c_int]
        L.fmm_plan_read_timing.argtypes = [vp, P(ctypes.c_double), P(i64)]
        L.fmm_plan_destroy.argtypes = [vp]
        L.fmm_plan_batch.argtypes = [i32, P(vp), P(i64), P(i32), P(i32), P(Options), P(Allocator), vp, i32,
                                     P(vp)]
        L.fmm_cached_bytes.argtypes = [ctypes.c_int, P(ctypes.c_size_t)]
        L.fmm_order_table.argtypes = [i32, i32, vp, i64, P(i64), P(i32)]
        L.fmm_last_error.restype = ctypes.c_char_p
        L.fmm_last_error.argtypes = []
        _lib = L
    return _lib


def _check(rc):
    if rc != FMM_OK:
        raise FmmError(rc, lib().fmm_last_error().decode())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


M2L_METHODS = {"sign_class": 0, "rotation": 1}
KERNELS = {"coulomb": 0, "softened": 1}


def _options(uniform_depth, max_depth, precision, want_field, root, m2l="sign_class", kernel="coulomb",
             softening=0.0):
    o = Options()
    lib().fmm_default_options(ctypes.byref(o))
    o.m2l_method = M2L_METHODS[m2l] if isinstance(m2l, str) else int(m2l)
    o.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.softening = float(softening)
    o.uniform_depth = uniform_depth
    o.max_depth = max_depth
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else precision
    o.want_field = 1 if want_field else 0
    keep = None
    if root is not None:
        keep = (ctypes.c_double * 4)(*[float(v) for v in root])
        o.root = ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
    return o, keep


class Plan:
    """Octree, interaction lists and workspace for one point set (fmm_plan)."""

    def __init__(self, xyz, order, leaf_size=64, uniform_depth=-1, max_depth=21,
                 precision="fp64", want_field=True, root=None, stream=None, allocator=None, m2l="sign_class",
                 kernel="coulomb", softening=0.0):
        """allocator: an Allocator (C function pointers) for the plan's device
        memory, or None for the library's own stream-ordered allocation.
        m2l: "sign_class" (matrix cores) or "rotation" (Sec. 3.4, vector unit).
        kernel: "coulomb" (1/r) or "softened" (1/sqrt(r^2 + softening^2);
        uniform trees, FP64, order <= 10)."""
        import torch
        if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda):
            raise FmmError(FMM_EINVAL, "xyz must be a CUDA/HIP tensor")
        xyz = xyz.to(torch.float64).contiguous()
        if xyz.dim() != 2 or xyz.shape[1] != 3:
            raise FmmError(FMM_EINVAL, "xyz must have shape [n, 3]")
        self.n = int(xyz.shape[0])
        self.order = int(order)
        self.device = xyz.device
        o, keep = _options(uniform_depth, max_depth, precision, want_field, root, m2l, kernel, softening)
        h = ctypes.c_void_p()
        _check(lib().fmm_plan(_ptr(xyz), self.n, self.order, int(leaf_size), ctypes.byref(o),
                              ctypes.byref(allocator) if allocator is not None else None,
                              _stream(stream), ctypes.byref(h)))
        self._h = h
        del keep

    @classmethod
    def _adopt(cls, h, n, order, device):
        self = cls.__new__(cls)
        self._h, self.n, self.order, self.device = h, int(n), int(order), device
        return self

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().fmm_plan_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def evaluate(self, q, phi=None, field=None, want_field=True, stream=None):
        import torch
        q = q.to(torch.float64).contiguous()
        if q.shape != (self.n,) or not q.is_cuda:
            raise FmmError(FMM_EINVAL, "q must be a device tensor of shape [n]")
        if phi is None:
            phi = torch.empty(self.n, dtype=torch.float64, device=q.device)
        if field is None and want_field:
            field = torch.empty(self.n, 3, dtype=torch.float64, device=q.device)
        _check(lib().fmm_evaluate(self._h, _ptr(q), _ptr(phi), _ptr(field), _stream(stream)))
        return phi, field

    def sizes(self):
        out = (ctypes.c_int64 * 10)()
        _check(lib().fmm_plan_sizes(self._h, out))
        keys = ["boxes", "U", "V", "W", "X", "depth", "key_depth", "n", "order", "ncoef"]
        return dict(zip(keys, [int(v) for v in out]))

    def footprint(self):
        b = ctypes.c_size_t()
        _check(lib().fmm_plan_footprint(self._h, ctypes.byref(b)))
        return int(b.value)

    def export_tree(self, stream=None):
        s = self.sizes()
        nb = s["boxes"]
        d = dict(root=np.zeros(4), perm=np.zeros(self.n, np.int64), level=np.zeros(nb, np.int32),
                 morton=np.zeros(nb, np.uint64), first=np.zeros(nb, np.int64), count=np.zeros(nb, np.int64),
                 parent=np.zeros(nb, np.int32), child_begin=np.zeros(nb, np.int32), nchild=np.zeros(nb, np.int32))
        for k in "UVWX":
            d[k + "_off"] = np.zeros(nb + 1, np.int64)
            d[k + "_src"] = np.zeros(max(s[k], 1), np.int32)
        keys = ["root", "perm", "level", "morton", "first", "count", "parent", "child_begin", "nchild",
                "U_off", "U_src", "V_off", "V_src", "W_off", "W_src", "X_off", "X_src"]
        _check(lib().fmm_plan_export_tree(self._h, _stream(stream),
                                          *[ctypes.c_void_p(d[k].ctypes.data) for k in keys]))
        for k in "UVWX":
            d[k + "_src"] = d[k + "_src"][:s[k]]
        return d

    def set_timing(self, on=True):
        _check(lib().fmm_plan_set_timing(self._h, 1 if on else 0))

    def read_timing(self):
        """{stage: (total ms, timed evaluations)} since the previous read."""
        ms = (ctypes.c_double * 16)()
        calls = (ctypes.c_int64 * 16)()
        _check(lib().fmm_plan_read_timing(self._h, ms, calls))
        return {name: (ms[i], int(calls[i])) for i, name in enumerate(STAGES)}

    def export_expansions(self, stream=None):
        s = self.sizes()
        M = np.zeros((s["boxes"], s["ncoef"]))
        L = np.zeros((s["boxes"], s["ncoef"]))
        _check(lib().fmm_plan_export_expansions(self._h, _stream(stream), ctypes.c_void_p(M.ctypes.data),
                                                ctypes.c_void_p(L.ctypes.data)))
        return M, L


def plan(xyz, order, leaf_size=64, **kw):
    return Plan(xyz, order, leaf_size, **kw)


def plan_batch(xyzs, orders, leaf_size=64, precision="fp64", uniform_depth=-1, max_depth=21,
               want_field=True, threads=8, stream=None):
    """fmm_plan_batch: build one plan per point set, concurrently on up to
    `threads` host threads; orders, leaf_size and precision may be scalars or
    per-problem sequences."""
    import torch
    m = len(xyzs)
    seq = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * m
    orders, leafs, precs = seq(orders), seq(leaf_size), seq(precision)
    xs = []
    for x in xyzs:
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dim() == 2 and x.shape[1] == 3):
            raise FmmError(FMM_EINVAL, "every xyz must be a CUDA/HIP tensor of shape [n, 3]")
        xs.append(x.to(torch.float64).contiguous())
    xv = (ctypes.c_void_p * m)(*[x.data_ptr() for x in xs])
    nv = (ctypes.c_int64 * m)(*[x.shape[0] for x in xs])
    ov = (ctypes.c_int32 * m)(*[int(o) for o in orders])
    lv = (ctypes.c_int32 * m)(*[int(l) for l in leafs])
    opts = (Options * m)()
    for i in range(m):
        opts[i], _ = _options(uniform_depth, max_depth, precs[i], want_field, None)
    hv = (ctypes.c_void_p * m)()
    _check(lib().fmm_plan_batch(m, xv, nv, ov, lv, opts, None, _stream(stream), int(threads), hv))
    return [Plan._adopt(ctypes.c_void_p(hv[i]), xs[i].shape[0], orders[i], xs[i].device) for i in range(m)]


def evaluate_batch(plans, qs, want_field=True, stream=None, noalloc=False):
    """One fmm_evaluate_batch call over several plans (fmm_evaluate_batch_noalloc
    with noalloc=True); returns [(phi, field)]."""
    import torch
    n = len(plans)
    outs = []
    qv = (ctypes.c_void_p * n)()
    pv = (ctypes.c_void_p * n)()
    fv = (ctypes.c_void_p * n)()
    hv = (ctypes.c_void_p * n)()
    keep = []
    for i, (p, q) in enumerate(zip(plans, qs)):
        q = q.to(torch.float64).contiguous()
        phi = torch.empty(p.n, dtype=torch.float64, device=q.device)
        fld = torch.empty(p.n, 3, dtype=torch.float64, device=q.device) if want_field else None
        keep.append(q)
        outs.append((phi, fld))
        qv[i] = q.data_ptr()
        pv[i] = phi.data_ptr()
        fv[i] = fld.data_ptr() if fld is not None else None
        hv[i] = p.handle.value
    fn = lib().fmm_evaluate_batch_noalloc if noalloc else lib().fmm_evaluate_batch
    _check(fn(hv, qv, pv, fv if want_field else None, n, _stream(stream)))
    return outs


def order_table(order, which):
    """fmm_order_table: one per-order constant table (host copy) as a 2-D array
    of rows of its leading dimension."""
    cnt, ld = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().fmm_order_table(int(order), int(which), None, 0, ctypes.byref(cnt), ctypes.byref(ld)))
    out = np.zeros(cnt.value)
    _check(lib().fmm_order_table(int(order), int(which), ctypes.c_void_p(out.ctypes.data), cnt.value,
                                 ctypes.byref(cnt), ctypes.byref(ld)))
    return out.reshape(-1, ld.value)


def cached_bytes(device=0):
    """Device bytes the library caches outside any plan (fmm_cached_bytes)."""
    b = ctypes.c_size_t()
    _check(lib().fmm_cached_bytes(int(device), ctypes.byref(b)))
    return int(b.value)


def estimate(n, order, leaf_size=64, uniform_depth=-1, max_depth=21, precision="fp64", kernel="coulomb"):
    o, keep = _options(uniform_depth, max_depth, precision, True, None, kernel=kernel)
    b = ctypes.c_size_t()
    _check(lib().fmm_plan_estimate(int(n), int(order), int(leaf_size), ctypes.byref(o), ctypes.byref(b)))
    return int(b.value)
