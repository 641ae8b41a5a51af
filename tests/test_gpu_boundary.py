"""Boundary of the C ABI on the GPU: non-finite coordinates are rejected by
fmm_plan with FMM_EINVAL, a caller's allocator serves every device
allocation of a plan and gets all of it back, and an allocator that fails
gives FMM_ENOMEM without leaking what it handed out."""
import ctypes

import numpy as np
import pytest

from paper_2508_02626_amd import inputs
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """fmm_allocator_t backed by torch's caching allocator; fails every
    request after the first `fail_after` (None: never)."""

    def __init__(self, fail_after=None):
        import torch
        from paper_2508_02626_amd import fmm
        self.torch = torch
        self.fail_after = fail_after
        self.live = {}
        self.calls = 0
        self.failed = 0
        self._a = ALLOC(self._alloc)
        self._f = FREE(self._free)
        self.c = fmm.Allocator(ctypes.cast(self._a, ctypes.c_void_p), ctypes.cast(self._f, ctypes.c_void_p), None)

    def _alloc(self, nbytes, stream, ctx):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            self.failed += 1
            return None
        ptr = self.torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0))
        self.live[ptr] = int(nbytes)
        return ptr

    def _free(self, ptr, stream, ctx):
        del self.live[ptr]
        self.torch.cuda.caching_allocator_delete(ptr)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_coordinates_rejected(bad):
    from paper_2508_02626_amd import fmm
    x, _ = inputs.uniform(5000, 3)
    x[1234, 1] = bad
    for kw in (dict(leaf_size=32), dict(uniform_depth=3)):
        with pytest.raises(fmm.FmmError) as e:
            fmm.Plan(to_dev(x), 6, **kw)
        assert e.value.code == fmm.FMM_EINVAL and "non-finite" in str(e.value), kw


def test_caller_allocator_serves_the_plan():
    from paper_2508_02626_amd import fmm
    x, q = inputs.plummer(40_000, 7)
    xd, qd = to_dev(x), to_dev(q)
    ref = fmm.Plan(xd, 8, leaf_size=32)
    a, fa = ref.evaluate(qd)
    ref.close()
    al = TorchAllocator()
    pl = fmm.Plan(xd, 8, leaf_size=32, allocator=al.c)
    b, fb = pl.evaluate(qd)
    assert al.calls > 0 and al.live
    assert pl.footprint() == sum(al.live.values())   # every owned byte came from the allocator
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert np.array_equal(fa.cpu().numpy(), fb.cpu().numpy())
    pl.close()
    al.torch.cuda.synchronize()
    say("  allocator calls %d, outstanding after destroy %d" % (al.calls, len(al.live)))
    assert not al.live


@pytest.mark.parametrize("fail_after", [0, 1, 3])
def test_failing_allocator_gives_enomem_without_leaks(fail_after):
    from paper_2508_02626_amd import fmm
    x, _ = inputs.plummer(40_000, 8)
    xd = to_dev(x)
    cached = fmm.cached_bytes(0)
    al = TorchAllocator(fail_after=fail_after)
    with pytest.raises(fmm.FmmError) as e:
        fmm.Plan(xd, 8, leaf_size=32, allocator=al.c)
    assert e.value.code == fmm.FMM_ENOMEM
    al.torch.cuda.synchronize()
    assert al.failed >= 1 and not al.live             # what it handed out came back
    assert fmm.cached_bytes(0) == cached               # the library's own cache untouched
    # the library still works afterwards
    pl = fmm.Plan(xd, 4, leaf_size=32)
    pl.close()
