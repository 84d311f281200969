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


def test_batch_bit_identical_to_plain(pcx, oracle_lib):
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


def test_batch_mixed_dims_output_fallback_and_degenerate(pcx, oracle_lib):
    nets = [wl.he_mlp([2, 12, 12, 1], 201), wl.he_mlp([3, 10, 10, 1], 202), wl.he_mlp([1, 9, 9, 9, 1], 203),
            wl.he_mlp([3, 64, 64, 64, 1], 5),          # too large for the batched kernel: per-step path
            wl.Net([2, 1, 1], [np.array([[1.0, 1.0]]), np.array([[1.0]])], [np.zeros(1), np.zeros(1)]),  # not generic
            wl.he_mlp([4, 6, 6, 1], 204), wl.he_mlp([2, 33, 70, 1], 205)]
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


def test_batch_full_workload_every_network(pcx, oracle_lib):
    """All 4096 networks of the batched workload in one launch: every network
    bit-identical to its per-step extraction (values and numbering) and equal
    to the oracle's complex in canonical form (signs and incidence exact,
    coordinates within 1e-10)."""
    from conftest import oracle_pool
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
        cx.close()
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b), f"network {i} differs from the per-step path"
        r = futs[i].result()
        futs[i] = None  # results are held only until checked
        X, SG, Ed = got
        assert_same_complex((X, unpack_signs(SG, net.widths), Ed), (r.X, r.S, r.edges))
        info = bt.info(i)
        assert (info.V, info.E, info.total_splits) == (r.V, r.E, int(r.steps[:, 2].sum()))
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
