"""Host-side serving policy (no GPU): admission in arrival order under a
memory budget, rejection of requests that can never fit or name an unknown
scene, cancellation, budget release."""
import pytest

from paper_2412_15867_amd.serve import ADMITTED, CANCELLED, QUEUED, REJECTED, Scheduler


def test_admission_respects_budget_and_order():
    s = Scheduler(n_scenes=3, budget_bytes=1000, bytes_per_ray=10)
    a = s.new_request(0, 50, arrival=0.0)
    b = s.new_request(1, 40, arrival=0.1)
    c = s.new_request(2, 30, arrival=0.2)
    got = s.admit(1.0)
    assert got == [a, b] and a.status == ADMITTED and c.status == QUEUED
    assert s.used == 900 and s.peak_used == 900
    assert s.admit(1.1) == []          # c does not fit until something is released
    s.release(a)
    assert s.admit(1.2) == [c]
    assert s.used == 700


def test_no_overtaking_of_a_large_request():
    s = Scheduler(1, 1000, 10)
    big = s.new_request(0, 90)
    small = s.new_request(0, 15)
    first = s.admit(0.0)
    assert first == [big]
    assert s.admit(0.0) == []          # small waits behind nothing but the budget
    s.release(big)
    assert s.admit(0.0) == [small]


def test_rejections_and_cancel():
    s = Scheduler(2, 1000, 10, max_launch_rays=80)
    assert s.new_request(5, 1).status == REJECTED
    assert s.new_request(0, 101).status == REJECTED     # larger than the budget
    assert s.new_request(0, 81).status == REJECTED      # larger than one launch
    assert s.new_request(0, -1).status == REJECTED
    r = s.new_request(1, 10)
    assert s.cancel(r) and r.status == CANCELLED
    assert not s.queue
    assert not s.cancel(r)


def test_launch_cap_splits_admission():
    s = Scheduler(1, 10**9, 1, max_launch_rays=100)
    reqs = [s.new_request(0, 40) for _ in range(5)]
    assert s.admit(0.0) == reqs[:2]
    assert s.admit(0.0) == reqs[2:4]
    assert s.admit(0.0) == reqs[4:]


def test_bad_budget():
    with pytest.raises(ValueError):
        Scheduler(1, 0, 10)
