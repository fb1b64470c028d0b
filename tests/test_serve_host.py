"""Host logic of the serving loop: admission by memory, in arrival order."""
import pytest

from paper_1904_07778_amd.serve import BLOCK_T, Admission, Request, realtime_period


def req(name, n, f, ring=4):
    return Request(name, n, f, dump_len=8192, n_dumps=1, ring_blocks=ring)


def test_footprint_counts_accumulator_dump_buffer_and_ring():
    r = req("a", 192, 1024)
    acc = 1024 * 18528 * 8
    assert r.footprint() == 2 * acc + 4 * BLOCK_T * 1024 * 192


def test_admission_in_order_under_budget():
    a, b, c = req("a", 192, 64), req("b", 32, 64), req("c", 96, 64)
    adm = Admission(a.footprint() + b.footprint())
    for r in (a, b, c):
        adm.submit(r)
    assert [r.name for r in adm.admit()] == ["a", "b"]
    assert adm.admit() == []                      # c waits: no room
    adm.release(b)
    assert adm.admit() == []                      # still no room for c
    adm.release(a)
    assert [r.name for r in adm.admit()] == ["c"]
    assert adm.used == c.footprint()


def test_head_of_line_is_not_overtaken():
    big, small = req("big", 192, 64), req("small", 16, 8)
    first = req("first", 96, 64)
    budget = max(big.footprint(), first.footprint() + small.footprint())
    assert first.footprint() + big.footprint() > budget
    adm = Admission(budget)
    adm.submit(first)
    adm.submit(big)
    adm.submit(small)
    assert [r.name for r in adm.admit()] == ["first"]   # big does not fit; small waits behind it
    adm.release(first)
    with pytest.raises(AssertionError):
        adm.release(first)


def test_request_larger_than_budget_is_refused():
    adm = Admission(1000)
    with pytest.raises(ValueError):
        adm.submit(req("huge", 192, 1024))


def test_realtime_period():
    # 1024 spectra of 1024 channels at 250 MSPS real sampling: 8.39 ms
    assert abs(realtime_period(1024) - 1024 * 2048 / 250e6) < 1e-12
    assert abs(realtime_period(256) - 2.097152e-3) < 1e-9
