"""Serving (continuous batching): requests that arrive while others run are
admitted as memory frees up and their work overlaps on the device; every
result must equal the one the same request gives alone (bit-identical)."""
import time

import numpy as np
import pytest

from checks import assert_same_complex, unpack_signs
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


def _predicted_vertices(D, N):
    # the order of magnitude of the complex (only picks which requests the oracle checks)
    f = 1.0
    for k in range(2, D):
        f *= 2.0 * k
    return 0.6 * N ** D / f


def test_served_workload_prefix_identical_alone_and_oracle(pcx, oracle_lib):
    """The first 64 requests of the served workload (D in {2,3}, widths 16-128,
    depths 2-4, the bench's seeds) arrive in bursts of sixteen, so many run
    together: batched ticks and per-step workers overlap on the device. Every
    result is bit-identical to the same request extracted alone, and every
    request whose complex is small enough for the oracle (about 100K vertices)
    equals the oracle's complex."""
    from conftest import oracle_pool
    reqs = wl.serve_requests(2000, rate_per_s=96.0)[:64]
    small = [i for i, r in enumerate(reqs)
             if _predicted_vertices(r.net.D, sum(r.net.widths[1:-1])) <= 1.0e5]
    assert len(small) >= 16
    pool = oracle_pool()
    futs = {i: pool.submit(oracle_lib.extract, reqs[i].net, reqs[i].box.lo, reqs[i].box.hi) for i in small}
    mlps = [pcx.MLP.from_net(r.net) for r in reqs]
    srv = pcx.Server()
    t0 = time.perf_counter()
    tickets = []
    for k, (r, m) in enumerate(zip(reqs, mlps)):
        # each burst at the arrival time of its first request
        dt = reqs[k - k % 16].arrival_s - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(m, r.box.lo, r.box.hi))
    res = [srv.wait(t) for t in tickets]
    assert all(x["status"] == 0 for x in res), [srv.error(t) for t in tickets if srv.wait(t)["status"]]
    nb = sum(x["batched"] for x in res)
    print(f"[serve] {nb} of {len(res)} requests ran in batched ticks; stats {srv.stats()}", flush=True)
    assert 0 < nb < len(res)
    checked = 0
    for i, (t, r, m) in enumerate(zip(tickets, reqs, mlps)):
        got = srv.copy(t)
        srv.release(t)
        cx = pcx.extract(m, r.box.lo, r.box.hi)
        ref = cx.copy()
        cx.close()
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b), f"request {i} differs from its alone extraction"
        if i in futs:
            o = futs.pop(i).result()
            X, SG, Ed = got
            assert_same_complex((X, unpack_signs(SG, r.net.widths), Ed), (o.X, o.S, o.edges))
            checked += 1
    print(f"[serve] {len(reqs)} results identical alone and in the mix; {checked} equal the oracle", flush=True)
    pool.shutdown()
    srv.close()
    for m in mlps:
        m.close()


def test_served_with_output_level_set_copy(pcx, oracle_lib):
    """A server that subdivides the output neuron too: copy() returns rows with
    the output's sign word (its sizes come from the server's result), equal to
    the same request alone and to the oracle."""
    archs = [(2, 16, 2), (3, 12, 2), (2, 24, 3), (3, 16, 3), (2, 40, 2), (2, 31, 4)]
    nets = [wl.he_mlp([D] + [w] * d + [1], [77, i]) for i, (D, w, d) in enumerate(archs)]
    mlps = [pcx.MLP.from_net(n) for n in nets]
    srv = pcx.Server(include_output=True)
    tickets = [srv.submit(m, wl.cube(n.D).lo, wl.cube(n.D).hi) for m, n in zip(mlps, nets)]
    for t, n, m in zip(tickets, nets, mlps):
        box = wl.cube(n.D)
        r = srv.wait(t)
        assert r["status"] == 0
        wd = 1 + sum((w + 31) // 32 for w in n.widths[1:])  # the output word included
        assert (r["D"], r["Wd"]) == (n.D, wd)
        X, SG, Ed = srv.copy(t)
        srv.release(t)
        assert SG.shape == (r["V"], wd)
        cx = pcx.extract(m, box.lo, box.hi, include_output=True)
        ref = cx.copy()
        cx.close()
        for a, b in zip((X, SG, Ed), ref):
            assert a.shape == b.shape and np.array_equal(a, b)
        o = oracle_lib.extract(n, box.lo, box.hi, include_output=True)
        assert_same_complex((X, unpack_signs(SG, n.widths, True), Ed), (o.X, o.S, o.edges))
    srv.close()
    for m in mlps:
        m.close()
