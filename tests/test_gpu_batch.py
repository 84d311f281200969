"""Batched extraction (one persistent launch for many networks): every
network's complex must be bit-identical to the per-step path's for the same
network (values and numbering), and equal to the oracle's in canonical form."""
import numpy as np
import pytest

from checks import assert_same_complex, unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def plain(pcx, net, box, incl=False):
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi, include_output=incl)
    out = cx.copy()
    cx.close()
    m.close()
    return out


def test_batch_bit_identical_to_plain(pcx, oracle_lib, monkeypatch):
    monkeypatch.setenv("PCX_NO_TINY", "1")  # the reference is the per-step kernels
    nets = wl.batch_nets(96)
    boxes = [(wl.cube(2).lo, wl.cube(2).hi)] * len(nets)
    mlps = [pcx.MLP.from_net(n) for n in nets]
    bt = pcx.Batch(mlps, boxes)
    st = bt.stats()
    assert st.n == 96 and st.degenerate == 0
    for i, net in enumerate(nets):
        got = bt.copy(i)
        ref = plain(pcx, net, wl.cube(2))
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b), f"network {i} differs from the per-step path"
        if i % 12 == 0:
            r = oracle_lib.extract(net, wl.cube(2).lo, wl.cube(2).hi)
            X, SG, Ed = got
            assert_same_complex((X, unpack_signs(SG, net.widths), Ed), (r.X, r.S, r.edges))
    bt.close()


@pytest.mark.parametrize("sched", [None, "4", "2"])  # tuned/default; 16 lanes per split; 64 lanes per split
def test_batch_mixed_dims_output_fallback_and_degenerate(pcx, oracle_lib, monkeypatch, sched):
    monkeypatch.setenv("PCX_NO_TINY", "1")  # the reference is the per-step kernels
    if sched is not None:
        monkeypatch.setenv("PCX_BATCH_SCHED", sched)
    nets = [wl.he_mlp([2, 12, 12, 1], 201), wl.he_mlp([3, 10, 10, 1], 202), wl.he_mlp([1, 9, 9, 9, 1], 203),
            wl.he_mlp([3, 64, 64, 64, 1], 5),          # too large for the batched kernel: per-step path
            wl.Net([2, 1, 1], [np.array([[1.0, 1.0]]), np.array([[1.0]])], [np.zeros(1), np.zeros(1)]),  # not generic
            wl.he_mlp([4, 6, 6, 1], 204), wl.he_mlp([2, 33, 70, 1], 205),
            wl.he_mlp([2, 96, 1], 206), wl.he_mlp([2, 140, 1], 207), wl.he_mlp([3, 20, 12, 1], 208)]
    boxes = [(wl.cube(n.D).lo, wl.cube(n.D).hi) for n in nets]
    mlps = [pcx.MLP.from_net(n) for n in nets]
    bt = pcx.Batch(mlps, boxes, include_output=True)
    st = bt.stats()
    assert st.degenerate == 1 and st.fallbacks >= 1
    for i, net in enumerate(nets):
        if i == 4:
            with pytest.raises(pcx.PcxError) as e:
                bt.info(i)
            assert e.value.code == pcx.PCX_ERR_DEGENERATE
            continue
        got = bt.copy(i)
        ref = plain(pcx, net, wl.cube(net.D), incl=True)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), f"network {i}"
        r = oracle_lib.extract(net, wl.cube(net.D).lo, wl.cube(net.D).hi, include_output=True)
        X, SG, Ed = got
        assert_same_complex((X, unpack_signs(SG, net.widths, True), Ed), (r.X, r.S, r.edges))
    bt.close()


def test_batch_full_workload_every_network(pcx, oracle_lib, monkeypatch):
    """All 4096 networks of the batched workload in one launch: every network
    bit-identical to its per-step extraction (values and numbering) and equal
    to the oracle's complex in canonical form (signs and incidence exact,
    coordinates within 1e-10)."""
    from conftest import oracle_pool
    monkeypatch.setenv("PCX_NO_TINY", "1")  # the reference is the per-step kernels
    nets = wl.batch_nets()
    box = wl.cube(2)
    pool = oracle_pool()
    futs = [pool.submit(oracle_lib.extract, n, box.lo, box.hi) for n in nets]
    mlps = [pcx.MLP.from_net(n) for n in nets]
    bt = pcx.Batch(mlps, [(box.lo, box.hi)] * len(nets))
    st = bt.stats()
    print(f"batch: {st}", flush=True)
    assert st.n == 4096 and st.degenerate == 0
    tot = [0, 0, 0]
    for i, net in enumerate(nets):
        got = bt.copy(i)
        cx = pcx.extract(mlps[i], box.lo, box.hi)
        ref = cx.copy()
        steps = cx.steps()
        cx.close()
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b), f"network {i} differs from the per-step path"
        r = futs[i].result()
        futs[i] = None  # results are held only until checked
        X, SG, Ed = got
        assert_same_complex((X, unpack_signs(SG, net.widths), Ed), (r.X, r.S, r.edges))
        info = bt.info(i)
        assert (info.V, info.E, info.total_splits) == (r.V, r.E, int(r.steps[:, 2].sum()))
        assert np.array_equal(bt.steps(i), r.steps), f"network {i}: per-step counters"
        assert np.array_equal(bt.steps(i), steps), f"network {i}: per-step counters vs the per-step path"
        tot[0] += r.V
        tot[1] += r.E
        tot[2] += int(r.steps[:, 2].sum())
        if i % 512 == 0:
            print(f"[batch] {i + 1}/4096 networks checked", flush=True)
    assert (st.total_V, st.total_E, st.total_splits) == tuple(tot)
    pool.shutdown()
    bt.close()
    for m in mlps:
        m.close()


def test_batch_schedules_and_tuner(pcx, monkeypatch):
    """Every launch schedule (lanes per splitting edge, edges per thread in the
    compaction) gives the same complexes, and the autotuner's choice is one of
    them, no slower than the default it was timed against."""
    monkeypatch.setenv("PCX_NO_TINY", "1")
    nets = wl.batch_nets(256)
    box = wl.cube(2)
    mlps = [pcx.MLP.from_net(n) for n in nets]
    boxes = [(box.lo, box.hi)] * len(nets)
    ref = None
    for sc in range(6):
        monkeypatch.setenv("PCX_BATCH_SCHED", str(sc))
        bt = pcx.Batch(mlps, boxes)
        st = bt.stats()
        assert (st.split_lanes, st.select_items) == (64 if sc & 2 else 16 if sc & 4 else 32, 8 if sc & 1 else 16)
        got = [bt.copy(i) for i in range(len(nets))]
        bt.close()
        if ref is None:
            ref = got
            continue
        for i, (a, b) in enumerate(zip(got, ref)):
            for x, y in zip(a, b):
                assert np.array_equal(x, y), f"schedule {sc}, network {i}"
    monkeypatch.delenv("PCX_BATCH_SCHED")
    t = pcx.batch_tune(mlps, boxes)
    print(f"tuned: {t}", flush=True)
    assert t["wg_per_cu"] in (1, 2, 4) and t["split_lanes"] in (16, 32, 64) and t["select_items"] in (8, 16)
    assert t["candidates"] == 8 and t["ms_best"] <= t["ms_default"]
    bt = pcx.Batch(mlps, boxes)
    st = bt.stats()
    assert (st.wg_per_cu, st.split_lanes, st.select_items) == (t["wg_per_cu"], t["split_lanes"], t["select_items"])
    for i in range(0, len(nets), 17):
        for x, y in zip(bt.copy(i), ref[i]):
            assert np.array_equal(x, y)
    bt.close()
