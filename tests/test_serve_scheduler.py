"""Host-side serving policy (no GPU): admission in arrival order under a
memory budget, rejection of requests that can never fit or name an unknown
scene, cancellation, budget release, splitting into work items and the turn
order that lets a small request ride in the next launch beside a large one,
and completion only when a request's last item has finished."""
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
    assert s.new_request(0, -1).status == REJECTED
    assert s.new_request(0, 81).status == QUEUED        # larger than one launch: split over several
    r = s.new_request(1, 10)
    assert s.cancel(r) and r.status == CANCELLED
    assert r not in s.queue
    assert not s.cancel(r)


def test_split_into_items_and_launch_cap():
    s = Scheduler(1, 10**9, 1, chunk_rays=30, max_launch_rays=100)
    r = s.new_request(0, 250)
    s.admit(0.0)
    l1 = s.next_launch()
    assert [(b, n) for _, b, n in l1] == [(0, 30), (30, 30), (60, 30), (90, 10)]
    l2 = s.next_launch()
    assert [(b, n) for _, b, n in l2] == [(100, 30), (130, 30), (160, 30), (190, 10)]
    l3 = s.next_launch()
    assert [(b, n) for _, b, n in l3] == [(200, 30), (230, 20)]
    assert s.next_launch() == []
    # completion only once every item has finished, in any order
    for it in l3 + l1:
        assert not s.item_done(r, it[2])
    done = [s.item_done(r, it[2]) for it in l2]
    assert done == [False, False, False, True]


def test_small_request_rides_in_the_next_launch():
    s = Scheduler(2, 10**9, 1, chunk_rays=64, max_launch_rays=256)
    big = s.new_request(0, 4096)
    s.admit(0.0)
    first = s.next_launch()
    assert all(r is big for r, _, _ in first)
    small = s.new_request(1, 10)
    s.admit(0.1)
    second = s.next_launch()
    assert small in [r for r, _, _ in second]
    assert sum(n for _, _, n in second) == 256
    # the small request finishes with that launch, long before the big one
    assert [s.item_done(r, n) for r, _, n in second if r is small] == [True]
    assert big.rays_left > 0


def test_turns_alternate_between_requests():
    s = Scheduler(1, 10**9, 1, chunk_rays=10, max_launch_rays=60)
    a = s.new_request(0, 100)
    b = s.new_request(0, 100)
    s.admit(0.0)
    order = [r for r, _, _ in s.next_launch()]
    assert order == [a, b, a, b, a, b]
    # no ray is placed twice and none is left out
    placed = {id(a): set(), id(b): set()}
    for it in [(r, bb, n) for r, bb, n in zip(order, [0, 0, 10, 10, 20, 20], [10] * 6)]:
        placed[id(it[0])].update(range(it[1], it[1] + it[2]))
    while True:
        items = s.next_launch()
        if not items:
            break
        for r, bb, n in items:
            rng = set(range(bb, bb + n))
            assert not (placed[id(r)] & rng)
            placed[id(r)] |= rng
    assert placed[id(a)] == set(range(100)) and placed[id(b)] == set(range(100))


def test_empty_request_completes():
    s = Scheduler(1, 100, 1)
    r = s.new_request(0, 0)
    s.admit(0.0)
    items = s.next_launch()
    assert items == [(r, 0, 0)]
    assert s.item_done(r, 0)


def test_bad_budget():
    with pytest.raises(ValueError):
        Scheduler(1, 0, 10)
    with pytest.raises(ValueError):
        Scheduler(1, 10, 10, chunk_rays=0)
