"""The serving scheduler on the CPU, with a test-double executor.

The double performs no arithmetic (a request's result is its input state), so
these tests cover scheduling only: admission under a device-memory budget,
back-pressure without drops, strict arrival order, per-request error
isolation, gate-chunked ticks, and disjoint arena regions.  Results of the
real GPU executor are checked in test_gpu_server.py.
"""
import threading

import numpy as np
import pytest

import qcw_inputs as qi
from paper_1101_1785_amd import _lib as L
from sched.harness import FakeServer, load

OK, EINVAL, EHIP, EAGAIN = 0, -1, -3, -4


@pytest.fixture(scope="module")
def lib():
    return load()


def _req(nq, G, seed):
    c = qi.circuit(seed, nq, G)
    gates, mats = L.pack_circuit(c)
    return gates, mats, qi.state(seed, nq, 5)


def test_every_request_completes(lib):
    s = FakeServer(lib)
    tickets = []
    for i in range(200):
        nq = 3 + i % 7
        g, m, p = _req(nq, 4 * nq, i)
        rc, t = s.submit(nq, g, m, p)
        assert rc == OK
        tickets.append((t, nq, p))
    for t, nq, p in tickets:
        rc, out, st = s.wait(t, nq)
        assert rc == OK and st.status == OK
        assert np.array_equal(out, p)
        assert st.t_submit_ns <= st.t_admit_ns <= st.t_done_ns
    c = s.counters()
    assert c.submitted == c.completed == 200 and c.rejected == 0
    assert s.violations() == 0
    rc, _, _ = s.poll(tickets[0][0], 3)        # released after the first successful read
    assert rc == EINVAL
    s.close()


def test_small_budget_backpressure_never_drops(lib):
    """A budget for ~2 requests: the rest wait, are admitted in arrival order,
    and all complete."""
    nq, G = 8, 32
    g, m, p = _req(nq, G, 1)
    from sched.harness import FakeServer as F
    need = (16 << nq) + 64 * G + 16 * m.size + 3 * 256
    s = F(lib, budget=2 * need, max_slots=16, tick_seconds=0.002)
    tickets = [s.submit(nq, g, m, p)[1] for _ in range(12)]
    done = []
    for t in tickets:
        rc, _, st = s.wait(t, nq)
        assert rc == OK
        done.append((st.t_admit_ns, st.t_done_ns, t))
    assert [t for (_, _, t) in sorted(done)] == tickets          # admitted in arrival order
    c = s.counters()
    assert c.completed == 12 and c.peak_active <= 2 and c.admit_waits > 0
    assert s.violations() == 0
    s.close()


def test_head_of_line_not_overtaken(lib):
    """A large request at the head is not overtaken by small ones behind it."""
    big = _req(10, 8, 2)
    small = _req(3, 4, 3)
    need_big = (16 << 10) + 64 * 8 + 16 * big[1].size + 3 * 256
    s = FakeServer(lib, budget=need_big + 4096, max_slots=8, tick_seconds=0.003)
    t_small0 = s.submit(3, *small)[1]
    t_big = s.submit(10, *big)[1]
    t_small = [s.submit(3, *small)[1] for _ in range(5)]
    _, _, st_big = s.wait(t_big, 10)
    for t in t_small:
        _, _, st = s.wait(t, 3)
        assert st.t_admit_ns >= st_big.t_admit_ns
    s.wait(t_small0, 3)
    assert s.violations() == 0
    s.close()


def test_max_slots_bounds_residency(lib):
    s = FakeServer(lib, max_slots=3, tick_seconds=0.001)
    g, m, p = _req(5, 20, 4)
    ts = [s.submit(5, g, m, p)[1] for _ in range(20)]
    for t in ts:
        assert s.wait(t, 5)[0] == OK
    assert s.counters().peak_active <= 3 and s.max_tick() <= 3
    s.close()


def test_invalid_requests_rejected_in_isolation(lib):
    s = FakeServer(lib, budget=1 << 16, max_nq=9)
    g, m, p = _req(4, 8, 5)
    bad = g.copy()
    bad[3]["q"][0] = 7                                           # target outside [1, 4]
    assert s.submit(4, bad, m, p)[0] == EINVAL
    assert b"gate 3" in lib.qcws_last_error()
    bad = g.copy()
    bad[0]["mat"] = m.size                                       # matrix outside mats
    assert s.submit(4, bad, m, p)[0] == EINVAL
    g10, m10, p10 = _req(10, 4, 6)
    assert s.submit(10, g10, m10, p10)[0] == EINVAL              # above max_nq
    gb, mb, pb = _req(9, 4, 7)
    s2 = FakeServer(lib, budget=4096, max_nq=11)
    assert s2.submit(9, gb, mb, pb)[0] == EINVAL                 # larger than the budget
    assert b"budget" in lib.qcws_last_error()
    s2.close()
    rc, t = s.submit(4, g, m, p)
    assert rc == OK and s.wait(t, 4)[0] == OK
    assert s.counters().rejected == 3
    s.close()


def test_upload_failure_isolated(lib):
    """A device error on one request's upload fails that request only."""
    g, m, p = _req(5, 10, 8)
    s = FakeServer(lib, fail_ticket=4, tick_seconds=0.001)
    ts = [s.submit(5, g, m, p)[1] for _ in range(8)]
    for t in ts:
        rc, out, st = s.wait(t, 5)
        if t == 4:
            assert rc == EHIP and st.status == EHIP
        else:
            assert rc == OK and np.array_equal(out, p)
    s.close()


@pytest.mark.parametrize("T,G,expect", [(0, 36, 1), (10, 36, 4), (36, 36, 1), (1, 5, 5),
                                        (7, 0, 1)])
def test_gate_chunked_ticks(lib, T, G, expect):
    s = FakeServer(lib, gates_per_tick=T)
    g, m, p = _req(6, G, 9) if G else (np.zeros(0, L.GATE_DTYPE), np.zeros(1, np.complex128),
                                         qi.state(9, 6))
    t = s.submit(6, g, m, p)[1]
    rc, _, st = s.wait(t, 6)
    assert rc == OK and st.ticks == expect
    s.close()


def test_concurrent_submitters(lib):
    s = FakeServer(lib, max_slots=32, tick_seconds=0.0005)
    results = {}

    def client(k):
        for i in range(40):
            nq = 3 + (k + i) % 6
            g, m, p = _req(nq, 2 * nq, 1000 * k + i)
            rc, t = s.submit(nq, g, m, p)
            assert rc == OK
            rc, out, _ = s.wait(t, nq)
            results[(k, i)] = rc == OK and np.array_equal(out, p)

    th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert len(results) == 240 and all(results.values())
    assert s.violations() == 0
    s.close()


def test_stop_fails_pending_without_hanging(lib):
    s = FakeServer(lib, max_slots=1, tick_seconds=0.01)
    g, m, p = _req(4, 4, 10)
    ts = [s.submit(4, g, m, p)[1] for _ in range(10)]
    s.stop()
    codes = [s.poll(t, 4)[0] for t in ts]
    assert all(c in (OK, EINVAL) for c in codes) and EINVAL in codes
    s.close()


def test_admission_overlaps_the_running_tick(lib):
    """A request that arrives while another request's tick runs is admitted
    (packed for upload) before that tick finishes, and runs in the tick right
    after it; gate ranges stay contiguous per slot (the double counts any
    break as a violation)."""
    s = FakeServer(lib, max_slots=8, gates_per_tick=3, tick_seconds=0.05)
    g, m, p = _req(5, 12, 11)
    rc, ta = s.submit(5, g, m, p)
    assert rc == OK
    import time
    time.sleep(0.02)                 # A's first tick (of four) is running
    rc, tb = s.submit(5, g, m, p)
    assert rc == OK
    ra, _, sa = s.wait(ta, 5)
    rb, _, sb = s.wait(tb, 5)
    assert ra == OK and rb == OK
    # A takes four ticks of 50 ms; B, admitted during A's first, finishes one
    # tick after A (not two: its first tick is launched right after A's first)
    assert sb.t_admit_ns < sa.t_admit_ns + 50_000_000
    assert sa.ticks == 4 and sb.ticks == 4
    assert sb.t_done_ns - sa.t_done_ns < 75_000_000
    assert s.violations() == 0
    s.close()
