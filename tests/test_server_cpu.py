"""Scheduling tests of the projector server on the CPU, with the simulated
executor (it computes nothing; a batch takes its output bytes / rate)."""
from __future__ import annotations

import threading
import time

import pytest

from paper_2510_05282_amd import _lib
from paper_2510_05282_amd.serve import (DONE, FAILED, PENDING, RELEASED, RUNNING, SH_F32, SH_F64, SH_REQ_AUTORELEASE,
                                        Server)

FAKE = 0x10000  # simulated atoms need a nonzero point address; it is never dereferenced


def _server(budget, **kw):
    kw.setdefault("sim_bytes_per_s", 1e10)
    return Server(budget, simulated=True, **kw)


def test_all_requests_complete_with_latencies():
    s = _server(1 << 30)
    a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=1000)
    b = s.add_atom(FAKE, [1, 1, 1], dtype=SH_F32, n=5000)
    tickets = [s.submit(a if k % 2 else b, k % 10, SH_REQ_AUTORELEASE) for k in range(200)]
    s.drain(30)
    st = s.stats()
    assert st["submitted"] == 200 and st["completed"] == 200 and st["failed"] == 0
    assert st["points_done"] == 100 * 1000 + 100 * 5000
    assert st["bytes_in_use"] == 0
    lat = s.latencies_ms()
    assert lat.shape == (200,) and (lat >= 0).all()
    assert all(s.poll(t) == RELEASED for t in tickets)
    s.close()


def test_budget_defers_admission():
    """Each output is 16*4096*8 = 512 KiB; a 1.2 MiB budget admits two at a time."""
    s = _server(int(1.2 * (1 << 20)), sim_bytes_per_s=2e8)
    a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=4096)
    for _ in range(12):
        s.submit(a, 3, SH_REQ_AUTORELEASE)
    s.drain(30)
    st = s.stats()
    assert st["completed"] == 12
    assert st["deferred"] >= 8
    assert st["peak_bytes"] <= int(1.2 * (1 << 20))
    s.close()


def test_results_hold_budget_until_released():
    s = _server(1 << 20, sim_bytes_per_s=1e12)
    a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=4096)  # 512 KiB at lmax 3
    t0 = s.submit(a, 3)
    t1 = s.submit(a, 3)
    t2 = s.submit(a, 3)
    assert s.wait(t0, 10) == DONE and s.wait(t1, 10) == DONE
    time.sleep(0.05)
    assert s.poll(t2) == PENDING  # no budget until a result is released
    p0, p1 = s.result_ptr(t0), s.result_ptr(t1)
    assert p0 != p1
    s.release(t0)
    assert s.wait(t2, 10) == DONE
    assert s.result_ptr(t2) == p0  # first fit reuses the freed block
    s.release(t1)
    s.release(t2)
    assert s.stats()["bytes_in_use"] == 0
    s.close()


def test_back_pressure_and_invalid_requests():
    s = _server(1 << 20, max_pending=4, sim_bytes_per_s=1e6)  # a batch takes about 0.5 s
    a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=4096)
    statuses = [s.try_submit(a, 3, SH_REQ_AUTORELEASE)[0] for _ in range(12)]
    assert 4 in statuses  # SH_EBUSY once max_pending requests wait
    assert s.try_submit(a, 10)[0] == 1  # lmax out of range
    assert s.try_submit(99, 3)[0] == 1  # unknown atom
    big = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=1 << 20)
    assert s.try_submit(big, 9)[0] == 1  # could never fit the budget
    s.close()  # shuts down with work outstanding, without hanging


def test_failed_batches_fail_only_their_requests():
    s = _server(1 << 30, sim_fail_every=3, n_slots=1)
    a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=1000)
    tickets = []
    for _ in range(30):
        tickets.append(s.submit(a, 2))
        s.wait(tickets[-1], 10)  # one request per batch
    states = [s.poll(t) for t in tickets]
    assert states.count(FAILED) == 10 and states.count(DONE) == 20
    st = s.stats()
    assert st["failed"] == 10 and st["completed"] == 20
    for t, state in zip(tickets, states):
        if state == DONE:
            s.release(t)
    assert s.stats()["bytes_in_use"] == 0
    with pytest.raises(_lib.ShError):
        s.result_ptr(tickets[2])
    s.close()


def test_concurrent_submitters():
    s = _server(1 << 30)
    a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F32, n=2000)
    got = [[] for _ in range(4)]

    def work(k):
        for _ in range(250):
            got[k].append(s.submit(a, 4, SH_REQ_AUTORELEASE))

    th = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    s.drain(30)
    all_t = sorted(t for g in got for t in g)
    assert all_t == list(range(1000))
    assert s.stats()["completed"] == 1000
    s.close()


def test_latency_includes_batch_time():
    """A lone request of B output bytes takes at least B / rate."""
    rate = 1e9
    s = _server(1 << 30, sim_bytes_per_s=rate)
    a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=100000)  # lmax 9: 80 MB -> 80 ms
    t = s.submit(a, 9, SH_REQ_AUTORELEASE)
    s.wait(t, 10)
    lat = s.latencies_ms()
    assert lat[0] >= 80.0 * 0.99
    s.close()


def test_small_request_completes_before_large_one_of_its_batch():
    """Requests complete as their part of a batch does, smallest output first: with
    one slot, a large (80 MB) and a small (8 KB) request queued behind a 20 MB one
    share the second batch; the small one completes right after the first batch,
    the large one 80 ms later."""
    rate = 1e9
    s = _server(1 << 30, n_slots=1, sim_bytes_per_s=rate)
    blocker = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=25000)  # lmax 9: 20 MB -> 20 ms
    big = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=100000)     # lmax 9: 80 MB -> 80 ms
    small = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=1000)     # lmax 0: 8 KB
    t0 = s.submit(blocker, 9, SH_REQ_AUTORELEASE)
    deadline = time.monotonic() + 5.0
    while s.poll(t0) < RUNNING:  # the first batch has been launched (it may have ended)
        assert time.monotonic() < deadline
        time.sleep(1e-4)
    s.submit(big, 9, SH_REQ_AUTORELEASE)
    s.submit(small, 0, SH_REQ_AUTORELEASE)
    s.drain(10)
    st = s.stats()
    assert st["completed"] == 3 and st["batches"] == 2, st
    lat = s.latencies_ms()  # completion order: blocker, small, big
    assert lat[1] < 40.0, lat
    assert lat[2] >= 80.0 * 0.99, lat
    s.close()


def test_drain_waits_for_batches_being_launched():
    """Regression: drain() must not return while the scheduler is launching a batch
    (a launch takes host time; the slot counts as busy from before it starts)."""
    for _ in range(5):
        s = _server(1 << 30, sim_launch_s=2e-3, sim_bytes_per_s=1e12)
        a = s.add_atom(FAKE, [0, 0, 0], dtype=SH_F64, n=1000)
        for k in range(60):
            s.submit(a, k % 10, SH_REQ_AUTORELEASE)
            if k % 7 == 0:
                time.sleep(1e-3)
        s.drain(30)
        st = s.stats()
        assert st["completed"] == 60, st
        s.close()


def test_atom_larger_than_one_batch_is_refused():
    """A batch is one dispatch: an atom whose tiles could not fit one batch grid is
    refused at registration (the simulated executor allows 2^22 tiles per batch)."""
    s = _server(1 << 30)
    limit = 256 * (1 << 22)
    assert s.add_atom(FAKE, [0, 0, 0], dtype=SH_F32, n=limit) >= 0
    with pytest.raises(_lib.ShError):
        s.add_atom(FAKE, [0, 0, 0], dtype=SH_F32, n=limit + 1)
    s.close()
