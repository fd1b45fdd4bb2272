"""Served meshing: every result equals the oracle's, and the same request
gives the same result alone and inside a concurrent mix (integer outputs:
tolerance zero)."""
import sys
import threading

import numpy as np
import pytest

import oracle
import paper_2403_14723_amd as gp
from paper_2403_14723_amd import workloads as W

pytestmark = pytest.mark.gpu
KEYS = ("next", "prev", "seeds", "loop_off", "loop_he")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests():
    out = [W.jittered_grid(n, seed=500 + n, warp=(n % 3 == 0)) for n in (1, 7, 30, 64, 99, 160, 257)]
    out += [W.random_delaunay(2000, 501), W.random_delaunay(15000, 502)]
    return out


@pytest.fixture(scope="module")
def ctx():
    c = gp.Context(0)
    yield c
    c.close()


def test_served_alone_equals_mix_and_oracle(ctx):
    reqs = _requests()
    with gp.Server(ctx, pool_bytes=2 << 30, max_batch=8, n_lanes=2) as srv:
        say("[gpu] serve: one at a time")
        alone = []
        for m in reqs:
            r = srv.wait(srv.submit(m.xy, m.tri))
            alone.append(r.copy())
            r.free()
        say("[gpu] serve: concurrent mix from two threads")
        tickets = [None] * len(reqs)

        def client(idx):
            for i in idx:
                tickets[i] = srv.submit(reqs[i].xy, reqs[i].tri)

        th = [threading.Thread(target=client, args=(range(k, len(reqs), 2),)) for k in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        mix = []
        for t in tickets:
            r = srv.wait(t, 60000)
            mix.append(r.copy())
            r.free()
        st = srv.stats()
    assert st["completed"] == 2 * len(reqs) and st["failed"] == 0
    for m, a, b in zip(reqs, alone, mix):
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (m.name, k)
        o = oracle.polylla(m.xy, m.tri)
        for k in KEYS:
            assert np.array_equal(a[k], getattr(o, k)), (m.name, k)


def test_served_errors(ctx):
    with gp.Server(ctx, pool_bytes=64 << 20, max_batch=4, n_lanes=1) as srv:
        say("[gpu] serve: bad request in a batch")
        bad = srv.submit(np.array([[0, 0], [1, 1], [2, 2]]), np.array([[0, 1, 2]]))
        good = W.jittered_grid(20, seed=9)
        ok = srv.submit(good.xy, good.tri)
        with pytest.raises(gp.GPolyllaError) as e:
            srv.wait(bad)
        assert e.value.code == gp.GP_EDEGEN
        r = srv.wait(ok)
        o = oracle.polylla(good.xy, good.tri)
        assert np.array_equal(r.copy()["loop_he"], o.loop_he)
        r.free()
        say("[gpu] serve: request larger than a lane")
        big = W.jittered_grid(1024, seed=1)
        with pytest.raises(gp.GPolyllaError) as e:
            srv.submit(big.xy, big.tri)
        assert e.value.code == gp.GP_ETOOBIG
        with pytest.raises(gp.GPolyllaError) as e:
            srv.wait(12345678, 10)
        assert e.value.code == gp.GP_EINVAL


def test_stop_drains_requests_in_flight(ctx):
    """Stopping a server with requests still queued and running finishes them
    all (each lane drains the queue before its thread ends); results never
    waited for are released by the stop."""
    reqs = [W.jittered_grid(n, seed=600 + n, warp=(n % 2 == 0)) for n in (40, 90, 150, 200, 64, 7, 128, 99)]
    srv = gp.Server(ctx, pool_bytes=1 << 30, max_batch=3, n_lanes=3)
    say("[gpu] serve: stop with requests in flight")
    first = srv.submit(reqs[0].xy, reqs[0].tri)
    r = srv.wait(first, 60000)
    o = oracle.polylla(reqs[0].xy, reqs[0].tri)
    assert np.array_equal(r.copy()["loop_he"], o.loop_he)
    r.free()
    for m in reqs * 4:
        srv.submit(m.xy, m.tri)
    st = srv.stats()
    assert st["submitted"] == 1 + 4 * len(reqs)
    srv.stop()   # returns once every lane has drained the queue


def test_reset_stats_with_requests_in_flight(ctx):
    """Statistics cleared while requests are queued or on a lane: those
    requests count as submitted afterwards, so once all are waited for,
    every one of them is completed and none is in flight."""
    reqs = [W.jittered_grid(n, seed=700 + n, warp=True) for n in (60, 120, 180, 240)]
    with gp.Server(ctx, pool_bytes=1 << 30, max_batch=2, n_lanes=2) as srv:
        say("[gpu] serve: reset_stats with requests in flight")
        tickets = [srv.submit(m.xy, m.tri) for m in reqs * 3]
        srv.reset_stats()
        mid = srv.stats()
        assert 0 <= mid["in_flight"] <= len(tickets)
        for t in tickets:
            srv.wait(t, 60000).free()
        st = srv.stats()
        assert st["failed"] == 0
        assert st["in_flight"] == 0
        assert st["completed"] == st["submitted"] == mid["in_flight"] + mid["completed"]


def test_queue_full_and_wait_timeout(ctx):
    """A full queue rejects a request with GP_EAGAIN and counts it; a wait
    that times out returns GP_ETIMEDOUT and leaves the ticket valid.  One lane
    and a queue of one: while the lane meshes a 2M-triangle request (a few
    milliseconds), tiny requests submitted back to back fill the queue."""
    big = W.jittered_grid(1024, seed=11)
    small = W.jittered_grid(6, seed=12)
    o = oracle.polylla(small.xy, small.tri)
    with gp.Server(ctx, pool_bytes=1 << 30, max_batch=1, max_queue=1, n_lanes=1) as srv:
        say("[gpu] serve: wait timeout and full queue")
        tb = srv.submit(big.xy, big.tri)
        with pytest.raises(gp.GPolyllaError) as e:
            srv.wait(tb, 0)
        assert e.value.code == gp.GP_ETIMEDOUT
        accepted, again = [], 0
        for _ in range(6):
            try:
                accepted.append(srv.submit(small.xy, small.tri))
            except gp.GPolyllaError as err:
                assert err.code == gp.GP_EAGAIN
                again += 1
        assert again >= 1
        r = srv.wait(tb, 60000)   # the ticket survived the timed-out wait
        assert r.info()["nt"] == big.nt
        r.free()
        for t in accepted:
            r = srv.wait(t, 60000)
            assert np.array_equal(r.copy()["loop_he"], o.loop_he)
            r.free()
        st = srv.stats()
        assert st["rejected"] == again
        assert st["completed"] == 1 + len(accepted) and st["failed"] == 0


def test_two_waiters_on_one_ticket(ctx):
    """Two threads wait for one ticket: one gets the result (equal to the
    oracle's), the other GP_EINVAL (the ticket is held by the first waiter,
    or already collected), and neither touches a freed request."""
    big = W.jittered_grid(1024, seed=13, warp=True)
    with gp.Server(ctx, pool_bytes=1 << 30, max_batch=1, n_lanes=1) as srv:
        say("[gpu] serve: two waiters on one ticket")
        t = srv.submit(big.xy, big.tri)
        got, errs = [], []

        def waiter():
            try:
                got.append(srv.wait(t, 60000))
            except gp.GPolyllaError as e:
                errs.append(e.code)

        th = [threading.Thread(target=waiter) for _ in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert len(got) == 1 and errs == [gp.GP_EINVAL]
        o = oracle.polylla(big.xy, big.tri)
        g = got[0].copy()
        got[0].free()
        for k in KEYS:
            assert np.array_equal(g[k], getattr(o, k)), k


def test_latency_runs_from_the_arrival(ctx):
    """A request submitted with an arrival 50 ms in the past reports a latency
    of at least 50 ms; an arrival in the future is refused; the result is the
    oracle's."""
    import time
    m = W.jittered_grid(20, seed=14)
    o = oracle.polylla(m.xy, m.tri)
    with gp.Server(ctx, pool_bytes=1 << 30, max_batch=4, n_lanes=1) as srv:
        say("[gpu] serve: latency from the arrival time")
        with pytest.raises(gp.GPolyllaError) as e:
            srv.submit(m.xy, m.tri, arrival_ns=time.monotonic_ns() + 10**9)
        assert e.value.code == gp.GP_EINVAL
        srv.reset_stats()
        t = srv.submit(m.xy, m.tri, arrival_ns=time.monotonic_ns() - 50 * 10**6)
        r = srv.wait(t, 60000)
        g = r.copy()
        r.free()
        for k in KEYS:
            assert np.array_equal(g[k], getattr(o, k)), k
        st = srv.stats()
        assert st["completed"] == 1 and st["p50_ms"] >= 50.0


def test_loops_only_results(ctx):
    """A loops-only server hands out the oracle's seeds and loops (Section 6.7:
    a polygon is its seed and the loop from it) and refuses a copy of
    next'/prev'; a mix of sizes across lanes keeps every block apart."""
    reqs = _requests()
    with gp.Server(ctx, pool_bytes=2 << 30, max_batch=4, n_lanes=2, loops_only=True) as srv:
        say("[gpu] serve: loops-only results")
        tickets = [srv.submit(m.xy, m.tri) for m in reqs]
        got = []
        for t in tickets:
            r = srv.wait(t, 60000)
            info = r.info()
            assert info["loops_only"] == 1
            nxt = np.empty(max(info["nh"], 1), np.int32)
            rc = gp._load().gpolylla_result_copy(r.handle, nxt.ctypes.data, None, None, None, None)
            assert rc == gp.GP_EINVAL
            got.append(r.copy())
            r.free()
    for m, g in zip(reqs, got):
        assert "next" not in g and "prev" not in g
        o = oracle.polylla(m.xy, m.tri)
        for k in ("seeds", "loop_off", "loop_he"):
            assert np.array_equal(g[k], getattr(o, k)), (m.name, k)
