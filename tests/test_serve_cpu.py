"""Host-side admission accounting of the serving loop (no GPU)."""
import threading

import pytest

from paper_2508_02626_amd.serve import Admission, order_for


def test_order_map():
    assert order_for(1e-4) == 4 and order_for(1e-7) == 8 and order_for(1e-9) == 12
    assert order_for(1e-3) == 4 and order_for(1e-12) == 12


def test_admission_reserves_and_refuses():
    a = Admission(1000)
    assert a.fits_alone(1000) and not a.fits_alone(1001)
    assert a.try_reserve(600)
    assert not a.try_reserve(500)        # would exceed the budget: must wait
    assert a.try_reserve(400)
    a.release(600)
    assert a.try_reserve(500)
    a.release(400)
    a.release(500)
    assert a.in_flight == 0
    with pytest.raises(AssertionError):
        a.release(1)


def test_admission_is_thread_safe():
    a = Admission(10_000)
    ok = []

    def worker():
        for _ in range(1000):
            if a.try_reserve(7):
                ok.append(1)
                a.release(7)
    ts = [threading.Thread(target=worker) for _ in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert a.in_flight == 0 and len(ok) == 8000


def test_precision_policy():
    from paper_2508_02626_amd.serve import precision_for
    # the mixed path only where its own error is far below the request
    assert precision_for(1e-4) == "mixed"
    assert precision_for(1e-7) == "fp64" and precision_for(1e-9) == "fp64"
