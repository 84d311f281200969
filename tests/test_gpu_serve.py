"""Serving (continuous batching): requests that arrive while others run are
admitted as memory frees up and their work overlaps on the device; every
result must equal the one the same request gives alone (bit-identical)."""
import time

import numpy as np
import pytest

from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def requests(n, seed, big_every=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        D = int(rng.choice([2, 3]))
        w = int(rng.integers(8, 41))
        d = int(rng.choice([2, 3]))
        if big_every and i % big_every == 0:
            D, w, d = 3, 48, 3   # above the batched kernel's threshold: per-step path
        out.append(wl.he_mlp([D] + [w] * d + [1], [seed, i]))
    return out


def alone(pcx, net):
    m = pcx.MLP.from_net(net)
    b = wl.cube(net.D)
    cx = pcx.extract(m, b.lo, b.hi)
    r = cx.copy()
    cx.close()
    m.close()
    return r


def test_results_identical_alone_and_in_the_mix(pcx):
    nets = requests(48, 301, big_every=16)
    mlps = [pcx.MLP.from_net(n) for n in nets]
    srv = pcx.Server(mem_budget=8 << 30, large_workers=2)
    tickets = [srv.submit(m, wl.cube(n.D).lo, wl.cube(n.D).hi) for m, n in zip(mlps, nets)]
    res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    nb = sum(r["batched"] for r in res)
    assert nb >= 24 and len(res) - nb >= 3  # both the batched ticks and the per-step workers served
    for t, net in zip(tickets, nets):
        got = srv.copy(t)
        ref = alone(pcx, net)
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b)
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == 48 and st["p50_ms"] <= st["p99_ms"]
    srv.close()


def test_poisson_stream_latency_stats(pcx):
    """Bursts of six arrivals spread over time (more than the per-step workers
    take at once): later requests are admitted while earlier ones run (several
    ticks), and every request completes."""
    nets = requests(60, 302)
    mlps = [pcx.MLP.from_net(n) for n in nets]
    rng = np.random.default_rng(5)
    arrivals = np.repeat(np.cumsum(rng.exponential(0.02, len(nets) // 6)), 6)
    srv = pcx.Server()
    t0 = time.perf_counter()
    tickets = []
    for a, m, n in zip(arrivals, mlps, nets):
        dt = a - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(m, wl.cube(n.D).lo, wl.cube(n.D).hi))
    res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    st = srv.stats()
    print("serve stats:", st)
    assert st["completed"] == 60 and st["ticks"] >= 2
    for t in tickets:
        srv.release(t)
    srv.close()


def test_lone_small_request_runs_on_a_free_worker(pcx):
    """A small request alone at an idle server goes to a per-step worker (a
    tick of one workgroup would answer later); the result is the same."""
    net = requests(1, 303)[0]
    m = pcx.MLP.from_net(net)
    srv = pcx.Server()
    t = srv.submit(m, wl.cube(net.D).lo, wl.cube(net.D).hi)
    r = srv.wait(t)
    assert r["status"] == 0 and r["batched"] == 0
    got = srv.copy(t)
    for a, b in zip(got, alone(pcx, net)):
        assert np.array_equal(a, b)
    srv.release(t)
    srv.close()
    m.close()
