"""Host logic of the serving loop: admission by slots and HBM bytes."""
import pytest

from paper_2406_09654_amd.serving import Admission


def test_fifo_admission_respects_bytes_and_slots():
    a = Admission(budget_bytes=100, max_worlds=3)
    for k, nb in enumerate([40, 30, 20, 10]):
        a.push(k, nb)
    assert a.pop_admissible() == [0, 1, 2]          # slots exhausted at 3
    assert a.used_bytes == 90 and a.used_slots == 3
    assert a.pop_admissible() == []
    a.release(40)
    assert a.pop_admissible() == [3]
    assert a.used_bytes == 60 and a.used_slots == 3


def test_backfill_is_bounded_so_the_head_cannot_starve():
    a = Admission(budget_bytes=100, max_worlds=100, max_bypass=2)
    a.push("big0", 90)
    assert a.pop_admissible() == ["big0"]
    a.push("big1", 60)                                 # blocked: 90 + 60 > 100
    for k in range(5):
        a.push("s%d" % k, 1)
    assert a.pop_admissible() == ["s0", "s1"]          # two may pass, then the head holds
    assert a.pop_admissible() == []
    a.release(90)
    assert a.pop_admissible() == ["big1", "s2", "s3", "s4"]
    assert a.bypass == 0 or a.bypass <= 2


def test_oversized_request_is_rejected():
    a = Admission(budget_bytes=10, max_worlds=4)
    with pytest.raises(ValueError):
        a.push("huge", 11)
    with pytest.raises(ValueError):
        Admission(0, 1)


def test_release_accounting_never_negative():
    a = Admission(budget_bytes=50, max_worlds=2)
    a.push(0, 50)
    assert a.pop_admissible() == [0]
    a.release(50)
    with pytest.raises(AssertionError):
        a.release(50)
