"""The exact pass of step 5 (Sec. 4.2.2: each splitting 2-face is met by
exactly two splitting edges, and pairs are found by comparing sign-vectors).

The hash paths only propose pairs: a 2-face word reached three times, a key
slot left without a partner, or equal hashes of different faces send the step
to the exact pass, which regroups the step's key slots by comparing their
2-face sign-vectors word by word. The test hooks PCX_DEBUG_HASH_BITS and
PCX_DEBUG_EXACT_BITS keep only a few bits of the hashes, so that collisions
happen in nearly every step: the complexes must not change (bit-identical to
the run without collisions, and equal to the oracle)."""
import numpy as np
import pytest

from checks import assert_same_complex, unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu

NETS = [
    ([2, 8, 8, 1], 1, False),
    ([2, 24, 24, 24, 1], 31, True),
    ([3, 12, 12, 1], 32, False),
    ([3, 20, 20, 1], 33, True),
    ([4, 7, 7, 1], 34, False),
    ([2, 70, 40, 1], 35, False),
]


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def run(pcx, net, incl, pairing="hash"):
    m = pcx.MLP.from_net(net)
    box = wl.cube(net.D)
    cx = pcx.extract(m, box.lo, box.hi, include_output=incl, pairing=pairing)
    out = cx.copy()
    info = cx.info()
    steps = cx.steps()
    cx.close()
    m.close()
    return out, info, steps


@pytest.mark.parametrize("widths,seed,incl", NETS)
def test_collisions_go_through_the_exact_pass(pcx, oracle_lib, monkeypatch, widths, seed, incl):
    net = wl.he_mlp(widths, seed)
    ref, info0, steps0 = run(pcx, net, incl)
    assert info0.exact_steps == 0
    monkeypatch.setenv("PCX_DEBUG_HASH_BITS", "2")
    monkeypatch.setenv("PCX_DEBUG_EXACT_BITS", "10")
    got, info, steps = run(pcx, net, incl)
    # with 2-bit hashes every face starts its probe at one of 4 words, all with the same key:
    # a step with more than four faces certainly pairs two different faces on the table
    busy = int((steps0[:, 3] > 8).sum())
    print(f"[exact] {widths}: {info.exact_steps} of {len(steps)} steps paired by the exact pass "
          f"({busy} with more than four pairs)", flush=True)
    assert info.exact_steps >= busy > 0
    for a, b in zip(got, ref):
        assert a.shape == b.shape and np.array_equal(a, b), "the exact pass changed the complex"
    assert np.array_equal(steps, steps0)
    # the sort mode's collisions (runs of equal 24-bit keys, equal 64-bit hashes) take the same pass;
    # with every busy step paired exactly, its edges come in the table path's order
    gs, infs, _ = run(pcx, net, incl, pairing="sort")
    assert infs.exact_steps > 0
    X, SG, Ed = gs
    box = wl.cube(net.D)
    r = oracle_lib.extract(net, box.lo, box.hi, include_output=incl)
    assert_same_complex((X, unpack_signs(SG, widths, incl), Ed), (r.X, r.S, r.edges))
    X, SG, Ed = got
    assert_same_complex((X, unpack_signs(SG, widths, incl), Ed), (r.X, r.S, r.edges))


def test_batched_collisions_retry_on_the_per_step_path(pcx, monkeypatch):
    """A pairing failure inside the batched kernel sends that network to the
    per-step path (whose exact pass tells a collision from a degenerate face):
    every network still comes out bit-identical to pcx_extract."""
    nets = wl.batch_nets(24)
    box = wl.cube(2)
    refs = [run(pcx, n, False)[0] for n in nets]
    monkeypatch.setenv("PCX_DEBUG_HASH_BITS", "2")
    monkeypatch.setenv("PCX_DEBUG_EXACT_BITS", "10")
    mlps = [pcx.MLP.from_net(n) for n in nets]
    bt = pcx.Batch(mlps, [(box.lo, box.hi)] * len(nets))
    st = bt.stats()
    assert st.degenerate == 0 and st.fallbacks > 0
    for i in range(len(nets)):
        for a, b in zip(bt.copy(i), refs[i]):
            assert a.shape == b.shape and np.array_equal(a, b), f"network {i}"
    bt.close()
    for m in mlps:
        m.close()


def test_exact_pass_on_the_large_workload_steps(pcx, monkeypatch):
    """The 768-neuron network on [-0.05, 0.05]^3 with 12-bit table hashes: the
    exact pass runs on steps of thousands of key slots and gives the same
    arrays."""
    net = wl.plain_large()
    lo, hi = np.full(3, -0.05), np.full(3, 0.05)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, lo, hi)
    ref = cx.copy()
    cx.close()
    monkeypatch.setenv("PCX_DEBUG_HASH_BITS", "12")
    cx = pcx.extract(m, lo, hi)
    got = cx.copy()
    info = cx.info()
    cx.close()
    m.close()
    print(f"[exact] large net: {info.exact_steps} of {info.n_steps} steps paired by the exact pass", flush=True)
    assert info.exact_steps > 100
    for a, b in zip(got, ref):
        assert a.shape == b.shape and np.array_equal(a, b)


@pytest.mark.parametrize("widths,seed,incl", NETS[:4])
def test_row_verification_changes_nothing(pcx, monkeypatch, widths, seed, incl):
    """verify_pairs (every hash-table pair's perturbed sign rows compared word
    by word) gives the same complex as the default, which relies on the
    mutual-record check; with collisions forced, both go through the exact
    pass alike."""
    net = wl.he_mlp(widths, seed)
    box = wl.cube(net.D)
    m = pcx.MLP.from_net(net)

    def go(verify):
        cx = pcx.extract(m, box.lo, box.hi, include_output=incl, verify_pairs=verify)
        out, info, steps = cx.copy(), cx.info(), cx.steps()
        cx.close()
        return out, info, steps

    monkeypatch.setenv("PCX_NO_TINY", "1")
    monkeypatch.setenv("PCX_NO_GRAPH", "1")
    a, ia, sa = go(False)
    b, ib, sb = go(True)
    assert ia.exact_steps == ib.exact_steps == 0
    assert all(np.array_equal(x, y) for x, y in zip(a, b)) and np.array_equal(sa, sb)
    monkeypatch.setenv("PCX_DEBUG_HASH_BITS", "2")
    c, ic, _ = go(False)
    d, id_, _ = go(True)
    assert ic.exact_steps > 0 and id_.exact_steps > 0
    assert all(np.array_equal(x, y) for x, y in zip(c, a)) and all(np.array_equal(x, y) for x, y in zip(d, a))
    monkeypatch.delenv("PCX_DEBUG_HASH_BITS")
    # the batched kernel, with and without the row comparison
    nets = [wl.he_mlp([2, w, w, 1], 600 + w) for w in (8, 16, 24, 32)]
    mlps = [pcx.MLP.from_net(n) for n in nets]
    boxes = [(wl.cube(2).lo, wl.cube(2).hi)] * len(nets)
    b0, b1 = pcx.Batch(mlps, boxes), pcx.Batch(mlps, boxes, verify_pairs=True)
    for i in range(len(nets)):
        assert all(np.array_equal(x, y) for x, y in zip(b0.copy(i), b1.copy(i)))
    b0.close()
    b1.close()
    for x in mlps:
        x.close()
    m.close()


def test_step_with_more_key_slots_than_24_bits_name(pcx):
    """6-32-32-1 on [-1,1]^6 (57M vertices): its largest steps have more than
    2^24 key slots, so the table words give the slot field more bits (and the
    key fewer); no step may fall back to the exact pass, and the per-step
    counters equal those of the sort pairing, which compares sign rows."""
    net = wl.he_mlp([6, 32, 32, 1], 6)
    box = wl.cube(6)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi)
    info, steps = cx.info(), cx.steps()
    cx.close()
    print(f"[exact] 6-32-32-1: V={info.V} E={info.E}, largest step {int(steps[:, 3].max())} paired key slots, "
          f"{info.exact_steps} exact steps", flush=True)
    assert int(steps[:, 2].max()) * 10 > (1 << 24)
    assert info.exact_steps == 0
    cx = pcx.extract(m, box.lo, box.hi, pairing="sort")
    s2 = cx.steps()
    cx.close()
    m.close()
    assert np.array_equal(steps, s2)
