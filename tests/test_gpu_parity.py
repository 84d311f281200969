"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact sign-vectors, vertex/edge counts, per-step counters and canonical
edge incidence; FP64 coordinates within 1e-10 (absolute).
"""
import json
import os

import numpy as np
import pytest

from checks import assert_same_complex, check_invariants, digest, unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def gpu_complex(pcx, net, box, include_output=False, **kw):
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi, include_output=include_output, **kw)
    X, SG, Ed = cx.copy()
    S = unpack_signs(SG, net.widths, include_output)
    steps = cx.steps()
    info = cx.info()
    cx.close()
    m.close()
    return X, S, Ed, steps, info


def _compare(oracle_lib, pcx, net, box, incl=False, invariants=True, pairing="hash"):
    X, S, Ed, steps, info = gpu_complex(pcx, net, box, incl, pairing=pairing)
    r = oracle_lib.extract(net, box.lo, box.hi, include_output=incl)
    assert info.V == r.V and info.E == r.E
    assert np.array_equal(steps, r.steps), "per-step counters differ"
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)
    if invariants:
        check_invariants(net, box.lo, box.hi, X, S, Ed, include_output=incl)
    return X, S, Ed


def test_plain_small_matches_oracle_and_golden(oracle_lib, pcx):
    net = wl.plain_small()
    box = wl.cube(2)
    X, S, Ed = _compare(oracle_lib, pcx, net, box)
    g = json.load(open(os.path.join(GOLDEN, "plain_small.json")))
    assert (len(X), len(Ed)) == (g["V"], g["E"])
    assert digest(S, Ed) == g["digest"]


@pytest.mark.parametrize("widths,seed,incl", [
    ([1, 9, 9, 1], 101, False),
    ([2, 16, 16, 16, 1], 102, False),
    ([2, 40, 33, 1], 103, True),
    ([3, 12, 12, 1], 104, False),
    ([3, 24, 20, 1], 105, True),
    ([4, 8, 8, 1], 106, False),
    ([2, 70, 1], 107, False),        # layer spanning three sign words
    ([3, 64, 1], 108, True),
    ([2, 1, 1, 1], 109, False),       # width-1 layers
    ([10, 9, 2, 1], 111, False),      # D = 10: splits with 18 key slots (more than a 16-lane group)
    ([3, 100, 1], 112, True),         # a layer of 65-128 neurons: 16-lane splits, 8 columns per lane
])
@pytest.mark.parametrize("pairing", ["hash", "sort"])
@pytest.mark.parametrize("path", ["default", "per-step"])
def test_small_nets_match_oracle(oracle_lib, pcx, monkeypatch, widths, seed, incl, pairing, path):
    # "default": the smallest of these networks take the batch of one (one launch of the batched kernel);
    # "per-step": every network on the per-step kernels
    if path == "per-step":
        monkeypatch.setenv("PCX_NO_TINY", "1")
    net = wl.he_mlp(widths, seed)
    _compare(oracle_lib, pcx, net, wl.cube(widths[0]), incl, pairing=pairing)


@pytest.mark.parametrize("widths,seed,incl", [([2, 8, 8, 1], 1, False), ([1, 9, 9, 1], 101, True),
                                              ([2, 1, 1, 1], 109, False), ([3, 5, 5, 1], 110, True),
                                              ([2, 12, 10, 1], 111, False)])
def test_batch_of_one_equals_the_per_step_path(pcx, monkeypatch, widths, seed, incl):
    """A small network's pcx_extract runs as a batch of one: the same arrays,
    numbering and per-step counters as the per-step kernels give."""
    net = wl.he_mlp(widths, seed)
    box = wl.cube(widths[0])
    m = pcx.MLP.from_net(net)
    out = []
    for off in ("0", "1"):
        monkeypatch.setenv("PCX_NO_TINY", off)
        cx = pcx.extract(m, box.lo, box.hi, include_output=incl)
        out.append((cx.copy(), cx.steps(), cx.info()))
        cx.close()
    m.close()
    (a, sa, ia), (b, sb, ib) = out
    for x, y in zip(a, b):
        assert x.shape == y.shape and np.array_equal(x, y)
    assert np.array_equal(sa, sb)
    assert (ia.V, ia.E, ia.total_splits, ia.total_pairs) == (ib.V, ib.E, ib.total_splits, ib.total_pairs)


def test_asymmetric_box(oracle_lib, pcx):
    net = wl.he_mlp([3, 10, 10, 1], 111)
    box = wl.Box(np.array([-0.7, -0.2, 0.1]), np.array([0.9, 0.5, 1.3]))
    _compare(oracle_lib, pcx, net, box)


def test_differentiable_small_matches_golden(oracle_lib, pcx):
    net = wl.differentiable_small()
    X, S, Ed = _compare(oracle_lib, pcx, net, wl.cube(3), incl=True)
    g = json.load(open(os.path.join(GOLDEN, "differentiable_small.json")))
    assert digest(S, Ed) == g["digest"]


@pytest.mark.parametrize("pairing", ["hash", "sort"])
def test_differentiable_workload_matches_oracle(oracle_lib, pcx, pairing):
    """3 -> 64 -> 64 -> 64 -> 1 with the output's zero level set: ~0.67M vertices."""
    net = wl.differentiable()
    box = wl.cube(3)
    X, S, Ed, steps, info = gpu_complex(pcx, net, box, True, pairing=pairing)
    g = json.load(open(os.path.join(GOLDEN, "differentiable.json")))
    assert (info.V, info.E) == (g["V"], g["E"])
    assert np.array_equal(steps, np.array(g["steps"]))
    assert digest(S, Ed) == g["digest"]
    r = oracle_lib.extract(net, box.lo, box.hi, include_output=True)
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)


@pytest.mark.parametrize("pairing", ["hash", "sort"])
def test_run_twice_bit_identical(pcx, pairing):
    net = wl.he_mlp([3, 32, 32, 1], 121)
    box = wl.cube(3)
    a = gpu_complex(pcx, net, box, pairing=pairing)
    b = gpu_complex(pcx, net, box, pairing=pairing)
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)


def test_no_subdivided_layer_is_the_box(pcx):
    net = wl.he_mlp([3, 1], 131)
    X, S, Ed, steps, info = gpu_complex(pcx, net, wl.cube(3))
    assert info.V == 8 and info.E == 12 and len(steps) == 0


def test_degenerate_input_is_reported(oracle_lib, pcx):
    """A hyperplane through two box corners is not generic (Sec. 3.2)."""
    net = wl.Net([2, 1, 1], [np.array([[1.0, 1.0]]), np.array([[1.0]])], [np.array([0.0]), np.array([0.0])])
    with pytest.raises(pcx.PcxError) as e:
        gpu_complex(pcx, net, wl.cube(2))
    assert e.value.code == pcx.PCX_ERR_DEGENERATE
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.extract(net, np.array([-1.0, -1.0]), np.array([1.0, 1.0]))


@pytest.mark.parametrize("pairing", ["hash", "sort"])
def test_storage_grown_by_redoing_steps(oracle_lib, pcx, monkeypatch, capfd, pairing):
    """With hash pairing the host runs ahead of the device; starting from
    the smallest storage, growing it happens after a step has found it too
    small, wrote nothing and is redone. The complex and the per-step counters
    are still the oracle's."""
    import re
    monkeypatch.setenv("PCX_VERBOSE", "1")
    monkeypatch.setenv("PCX_SMALL_START", "1")
    net = wl.he_mlp([3, 24, 24, 24], 77)
    capfd.readouterr()
    _compare(oracle_lib, pcx, net, wl.cube(3), incl=False, pairing=pairing)
    err = capfd.readouterr().err
    m = re.search(r"steps redone after growing the storage: (\d+)", err)
    assert m, err[-2000:]
    if pairing == "hash":
        assert int(m.group(1)) > 0
    else:
        assert int(m.group(1)) == 0  # sort pairing sizes every step exactly


def test_byte_cap_that_fits_the_complex(oracle_lib, pcx):
    """A byte cap at four times what an extraction used succeeds with the same
    complex on a fresh network (no capacity hints), and one below it fails
    cleanly with PCX_ERR_CAPACITY."""
    net = wl.he_mlp([3, 20, 20, 1], 131)
    box = wl.cube(3)
    X, S, Ed, steps, info = gpu_complex(pcx, net, box)
    cap = 4 * info.peak_bytes
    X2, S2, Ed2, steps2, info2 = gpu_complex(pcx, net, box, max_bytes=cap)
    assert info2.peak_bytes <= cap
    assert np.array_equal(steps, steps2)
    r = oracle_lib.extract(net, box.lo, box.hi)
    assert_same_complex((X2, S2, Ed2), (r.X, r.S, r.edges), coord_tol=1e-10)
    with pytest.raises(pcx.PcxError) as e:
        gpu_complex(pcx, net, box, max_bytes=info.peak_bytes // 8)
    assert e.value.code == pcx.PCX_ERR_CAPACITY


def test_vertex_on_two_hyperplanes_is_reported(oracle_lib, pcx):
    """A new vertex that lands exactly on a later neuron's hyperplane is not
    generic either: x = 0.5 cuts the bottom edge at (0.5, -1), where the
    second neuron x + y + 0.5 interpolates to exactly 0 (Sec. 3.2)."""
    net = wl.Net([2, 2, 1], [np.array([[1.0, 0.0], [1.0, 1.0]]), np.array([[1.0, 1.0]])],
                 [np.array([-0.5, 0.5]), np.array([0.0])])
    with pytest.raises(pcx.PcxError) as e:
        gpu_complex(pcx, net, wl.cube(2))
    assert e.value.code == pcx.PCX_ERR_DEGENERATE
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.extract(net, np.array([-1.0, -1.0]), np.array([1.0, 1.0]))


def test_invalid_arguments(pcx):
    net = wl.plain_small()
    m = pcx.MLP.from_net(net)
    with pytest.raises(pcx.PcxError) as e:
        pcx.extract(m, np.array([1.0, 0.0]), np.array([1.0, 1.0]))
    assert e.value.code == pcx.PCX_ERR_INVALID
    with pytest.raises(pcx.PcxError) as e:
        pcx.extract(m, np.array([-1.0, -1.0]), np.array([1.0, 1.0]), max_bytes=4096)
    assert e.value.code == pcx.PCX_ERR_CAPACITY
    wide = wl.he_mlp([2, 300, 1], 1)
    mw = pcx.MLP.from_net(wide)
    with pytest.raises(pcx.PcxError) as e:
        pcx.extract(mw, np.array([-1.0, -1.0]), np.array([1.0, 1.0]))
    assert e.value.code == pcx.PCX_ERR_INVALID


@pytest.mark.parametrize("pairing", ["hash", "sort"])
def test_kernel_timing_leaves_the_complex_unchanged(pcx, pairing):
    """Timed extractions (split launches record their own events, the other
    families sit between event markers) give the same bits; every neuron
    step's split launch is timed, and untimed families report nothing."""
    net = wl.he_mlp([3, 24, 20, 1], 105)
    box = wl.cube(3)
    m = pcx.MLP.from_net(net)
    ref = None
    try:
        for timing in (0, ["split"], True):
            cx = pcx.extract(m, box.lo, box.hi, timing=timing, pairing=pairing)
            got = cx.copy() + (cx.steps(),)
            times = {f: cx.kernel_time(f) for f in pcx.KERNEL_FAMILIES}
            cx.close()
            if ref is None:
                ref = got
                assert all(n == 0 for _, n in times.values())
                continue
            for a, b in zip(got, ref):
                assert np.array_equal(a, b)
            ms, n = times["split"]
            assert n >= 44 and ms > 0.0  # one launch per neuron step (redone steps add more)
            if timing != True:  # noqa: E712
                assert all(times[f][1] == 0 for f in pcx.KERNEL_FAMILIES if f != "split")
            else:
                assert times["gemm"][1] >= 2 and times["gemm"][0] > 0.0
    finally:
        m.close()


def _corner_net():
    """16 inputs (the box entries fill sign word 0): two hyperplanes cutting
    the corners (1,...,1) and (1,...,1,-1) of [-1,1]^16, then one neuron
    h1 + h2 = 0.2 inside the first corner."""
    w1 = np.ones((2, 16))
    w1[1, 15] = -1.0
    return wl.Net([16, 2, 1, 1], [w1, np.array([[1.0, 1.0]]), np.array([[1.0]])],
                  [np.array([-15.5, -15.3]), np.array([-0.2]), np.array([0.0])])


@pytest.mark.parametrize("pairing", ["hash", "sort"])
def test_sixteen_inputs_fill_the_box_word(oracle_lib, pcx, pairing):
    """D = 16, the largest input dimension: 65,536 corners, 524,288 box edges,
    30 key slots per split (2-faces at a box corner), every box entry in word 0."""
    net = _corner_net()
    box = wl.cube(16)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi, pairing=pairing)
    X, SG, Ed = cx.copy()
    steps = cx.steps()
    cx.close()
    m.close()
    r = oracle_lib.extract(net, box.lo, box.hi)
    assert np.array_equal(steps, r.steps)
    assert_same_complex((X, unpack_signs(SG, net.widths), Ed), (r.X, r.S, r.edges))


def test_empty_batch_and_idle_server(pcx):
    """A batch of no networks and a server that never gets a request."""
    bt = pcx.Batch([], [])
    st = bt.stats()
    assert st.n == 0 and st.total_V == 0 and st.fallbacks == 0
    bt.close()
    srv = pcx.Server()
    s = srv.stats()
    assert s["completed"] == 0
    srv.close()
