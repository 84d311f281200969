"""Repeated extractions of one network replay a captured HIP graph: the
network's first extraction records its step log, the next one captures the
whole kernel sequence, later ones replay it. Every replay must give the
complex the ordinary path gives (bit-identical arrays and counters), with the
program's own eager work and synchronisations between the replays."""
import numpy as np
import pytest

from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def run(pcx, m, lo, hi, incl):
    cx = pcx.extract(m, lo, hi, include_output=incl)
    out = cx.copy()
    steps = cx.steps()
    info = cx.info()
    cx.close()
    return out, steps, info


def same(a, b):
    (oa, sa, ia), (ob, sb, ib) = a, b
    assert all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(oa, ob)), "arrays differ"
    assert np.array_equal(sa, sb)
    assert (ia.V, ia.E, ia.total_splits, ia.total_pairs) == (ib.V, ib.E, ib.total_splits, ib.total_pairs)


@pytest.mark.parametrize("name,incl", [("plain_small", False), ("differentiable_small", True),
                                       ("differentiable", True)])
def test_replays_equal_the_ordinary_path(pcx, monkeypatch, name, incl):
    monkeypatch.setenv("PCX_NO_TINY", "1")  # the smallest network would take the batch of one
    net = getattr(wl, name)()
    box = wl.cube(net.D)
    other = wl.he_mlp([2, 12, 12, 1], 91)
    mo = pcx.MLP.from_net(other)
    monkeypatch.setenv("PCX_NO_GRAPH", "1")
    m = pcx.MLP.from_net(net)
    ref = run(pcx, m, box.lo, box.hi, incl)
    ref_other = run(pcx, mo, wl.cube(2).lo, wl.cube(2).hi, False)
    m.close()
    monkeypatch.delenv("PCX_NO_GRAPH")
    m = pcx.MLP.from_net(net)
    for _ in range(2):  # the first two requests run on the ordinary path
        first = run(pcx, m, box.lo, box.hi, incl)
        assert first[2].from_graph == 0
        same(first, ref)
    for k in range(5):
        r = run(pcx, m, box.lo, box.hi, incl)
        assert r[2].from_graph == 1, f"replay {k} did not come from the graph"
        same(r, ref)
        # eager work of the program between replays (another network, graph off)
        monkeypatch.setenv("PCX_NO_GRAPH", "1")
        same(run(pcx, mo, wl.cube(2).lo, wl.cube(2).hi, False), ref_other)
        monkeypatch.delenv("PCX_NO_GRAPH")
    # another box: the ordinary path first (a new log), then its own graph
    lo2, hi2 = box.lo * 0.5, box.hi * 0.5
    r1 = run(pcx, m, lo2, hi2, incl)
    r2 = run(pcx, m, lo2, hi2, incl)
    r3 = run(pcx, m, lo2, hi2, incl)
    assert (r1[2].from_graph, r2[2].from_graph, r3[2].from_graph) == (0, 0, 1)
    same(r2, r1)
    same(r3, r1)
    m.close()
    mo.close()


def test_capture_alongside_other_threads(pcx, monkeypatch):
    """A capture on one thread while other threads create and free networks,
    extract (per-step path and batched kernel) and copy results: every call
    succeeds and every result equals its reference. (The library puts nothing
    on the legacy default stream, and its allocations and frees wait for a
    capture in progress.)"""
    import threading
    monkeypatch.setenv("PCX_NO_TINY", "1")
    net = wl.differentiable()
    box = wl.cube(3)
    smalls = [wl.he_mlp([2, 16, 16, 1], 300 + i) for i in range(6)]
    sbox = wl.cube(2)
    monkeypatch.setenv("PCX_NO_GRAPH", "1")
    m = pcx.MLP.from_net(net)
    ref = run(pcx, m, box.lo, box.hi, True)
    refs = []
    for n in smalls:
        ms = pcx.MLP.from_net(n)
        refs.append(run(pcx, ms, sbox.lo, sbox.hi, False))
        ms.close()
    monkeypatch.delenv("PCX_NO_GRAPH")
    errors, got_graph = [], []

    def repeated():
        try:
            for _ in range(6):
                r = run(pcx, m, box.lo, box.hi, True)
                same(r, ref)
                got_graph.append(r[2].from_graph)
        except Exception as e:  # noqa: BLE001 - reported by the main thread
            errors.append(("repeated", repr(e)))

    def others(k):
        try:
            for it in range(8):
                i = (k + it) % len(smalls)
                ms = pcx.MLP.from_net(smalls[i])
                same(run(pcx, ms, sbox.lo, sbox.hi, False), refs[i])
                bt = pcx.Batch([ms, ms], [(sbox.lo, sbox.hi)] * 2)
                for j in range(2):
                    for x, y in zip(bt.copy(j), refs[i][0]):
                        assert np.array_equal(x, y)
                bt.close()
                ms.close()
        except Exception as e:  # noqa: BLE001
            errors.append((f"others {k}", repr(e)))

    ths = [threading.Thread(target=repeated)] + [threading.Thread(target=others, args=(k,)) for k in range(3)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    m.close()
    assert not errors, errors
    assert got_graph[:2] == [0, 0]
    print(f"replays from the graph: {got_graph}", flush=True)
