"""fmm_evaluate_batch_noalloc (the batched evaluation that allocates nothing,
its per-plan views staged in the library's fixed device array) against
fmm_evaluate_batch, through the C ABI: bitwise equal on two calls in a row,
the second with fewer and smaller plans; sizes beyond the array's limit are
rejected before any device work."""
import ctypes

import numpy as np
import pytest

from paper_2508_02626_amd import inputs
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _problems(specs):
    out = []
    for kind, n, seed, p, kw in specs:
        x, q = getattr(inputs, kind)(n, seed)
        out.append((x, q, p, kw))
    return out


def _run(problems, noalloc):
    from paper_2508_02626_amd import fmm
    plans = [fmm.Plan(to_dev(x), p, **kw) for x, q, p, kw in problems]
    qs = [to_dev(q) for _, q, _, _ in problems]
    outs = fmm.evaluate_batch(plans, qs, noalloc=noalloc)
    res = [(a.cpu().numpy(), b.cpu().numpy()) for a, b in outs]
    for pl in plans:
        pl.close()
    return res


def test_noalloc_batch_equals_allocating_batch_twice():
    first = _problems([
        ("plummer", 30_000, 31, 8, dict(leaf_size=32)),
        ("uniform", 20_000, 32, 6, dict(leaf_size=16, precision="mixed")),
        ("clusters", 15_000, 33, 12, dict(leaf_size=24)),
        ("uniform", 4000, 34, 4, dict(uniform_depth=3, root=[0, 0, 0, 1])),
        ("plummer", 9000, 35, 10, dict(leaf_size=64, precision="mixed")),
    ])
    second = _problems([   # fewer and smaller plans: the array keeps the first call's contents
        ("plummer", 3000, 36, 8, dict(leaf_size=32)),
        ("uniform", 1500, 37, 5, dict(leaf_size=16)),
    ])
    for i, probs in enumerate((first, second)):
        ref = _run(probs, noalloc=False)
        got = _run(probs, noalloc=True)
        for (a, fa), (b, fb) in zip(ref, got):
            assert np.array_equal(a, b) and np.array_equal(fa, fb)
        say("  noalloc call %d: %d plans bitwise equal" % (i + 1, len(probs)))


def test_noalloc_rejects_oversized_batches():
    from paper_2508_02626_amd import fmm
    L = fmm.lib()
    n = 1025
    arr = (ctypes.c_void_p * n)()
    rc = L.fmm_evaluate_batch_noalloc(arr, arr, arr, None, n, None)
    assert rc == fmm.FMM_EINVAL and b"1024" in L.fmm_last_error()
    assert L.fmm_evaluate_batch_noalloc(None, None, None, None, 0, None) == fmm.FMM_OK
    assert L.fmm_evaluate_batch_noalloc(None, None, None, None, -1, None) == fmm.FMM_EINVAL
