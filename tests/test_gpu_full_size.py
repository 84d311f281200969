"""Parity at the full size of the 768-neuron workload (MLP 3-256-256-256-1, seed 2,
box [-1, 1]^3: 3.8e7 vertices, 1.1e8 edges), run as the benchmark runs it (hash
pairing, no tape).

The oracle cannot subdivide all 768 neurons within a test, so the full run is
checked by parts the oracle or the mathematics fix exactly:

* the first layer alone (1.9e6 vertices) element by element against the oracle;
* the full run's per-step counters of its first 256 steps against the oracle's
  first-layer counters, and the first-layer totals against the closed-form count
  of the plane arrangement;
* per-step identities at every step: a split adds one vertex and one edge, a
  pair of keys one edge;
* on the packed rows of every vertex: D zeros, valid codes, box entries
  non-negative, box coordinates exact, rows distinct; degree 2D - z_box for every
  vertex (Sec. 4.1 at k = 0);
* on sampled edges: D - 1 shared zeros, no +/- conflict, midpoint in the edge's
  cell (Sec. 3.5, 4.2.2);
* on sampled vertices: the oracle's solve from the sign-vector lands on the same
  point, and the oracle's forward pass at the point reproduces the sign-vector.

Whole-complex comparisons of the same network run on centred sub-boxes: the
largest, [-0.125, 0.125]^3 (3.0M edges), also in the launch shape of the big
steps (every grid at its maximum).
"""
import numpy as np
import pytest

import brute
from checks import assert_same_complex, check_invariants, unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu

MASK01 = np.uint64(0x5555555555555555)


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def _word_masks(widths):
    """Per word of a packed row: the low bit of every used 2-bit field, and the
    low bits of the box fields (word 0)."""
    D = widths[0]
    nsub = len(widths) - 2
    words = [sum(1 << (2 * e) for e in range(2 * D))]
    for l in range(1, nsub + 1):
        n = widths[l]
        for w in range(-(-n // 32)):
            k = min(32, n - 32 * w)
            words.append(sum(1 << (2 * f) for f in range(k)))
    used = np.array(words, np.uint64)
    return used, used[0]


def _zeros_per_row(SG, used):
    nz = (SG | (SG >> np.uint64(1))) & MASK01
    return np.bitwise_count(used & ~nz).sum(axis=1, dtype=np.int64)


@pytest.fixture(scope="module")
def full(pcx):
    net = wl.plain_large()
    box = wl.cube(3)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi, pairing="hash")
    info = cx.info()
    steps = cx.steps().astype(np.int64)
    X, SG, Ed = cx.copy()
    cx.close()
    m.close()
    print(f"[full] V={info.V} E={info.E} splits={info.total_splits}", flush=True)
    return net, box, info, steps, X, SG, Ed


def test_first_layer_alone_matches_oracle(oracle_lib, pcx):
    """Layer 1 of the workload as its own network: 1.87M vertices, element by element."""
    big = wl.plain_large()
    net = wl.Net([3, 256, 1], [big.W[0], np.zeros((1, 256))], [big.b[0], np.zeros(1)], "plain_large_layer1")
    box = wl.cube(3)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi)
    X, SG, Ed = cx.copy()
    steps = cx.steps()
    cx.close()
    m.close()
    S = unpack_signs(SG, net.widths)
    r = oracle_lib.extract(net, box.lo, box.hi)
    assert (len(X), len(Ed)) == (r.V, r.E) == brute.arrangement_counts_3d(net.W[0], net.b[0], box.lo, box.hi)
    assert np.array_equal(steps, r.steps)
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)


def test_full_counters(oracle_lib, full):
    net, box, info, steps, X, SG, Ed = full
    assert steps.shape == (768, 4)
    # per-step identities: a split adds one vertex and one edge; two keys make one intersecting edge
    V, E, S, K = steps.T
    assert np.all(K % 2 == 0)
    assert np.array_equal(V[1:], V[:-1] + S[:-1]) and np.array_equal(E[1:], E[:-1] + S[:-1] + K[:-1] // 2)
    assert info.V == V[-1] + S[-1] and info.E == E[-1] + S[-1] + K[-1] // 2
    assert info.total_splits == S.sum() and info.total_pairs == K.sum() // 2
    assert (len(X), len(Ed)) == (info.V, info.E)
    # the first layer: the oracle's counters step by step, and the closed-form arrangement count
    l1 = wl.Net([3, 256, 1], [net.W[0], np.zeros((1, 256))], [net.b[0], np.zeros(1)], "layer1")
    r = oracle_lib.extract(l1, box.lo, box.hi)
    assert np.array_equal(steps[:256], r.steps)
    assert (V[256], E[256]) == (r.V, r.E) == brute.arrangement_counts_3d(net.W[0], net.b[0], box.lo, box.hi)


def test_full_vertex_rows(full):
    net, box, info, steps, X, SG, Ed = full
    D = 3
    used, ubox = _word_masks(net.widths)
    assert SG.shape == (info.V, len(used))
    zbox = np.empty(info.V, np.int64)
    keys = np.empty(info.V, np.uint64)
    mult = np.random.default_rng(7).integers(1, 2 ** 63, len(used), dtype=np.uint64) | np.uint64(1)
    chunk = 1 << 21
    for s0 in range(0, info.V, chunk):
        R = SG[s0:s0 + chunk]
        x = X[s0:s0 + chunk]
        assert np.all(_zeros_per_row(R, used) == D), "vertex without exactly D zeros"
        assert not np.any(R & (R >> np.uint64(1)) & MASK01), "invalid code 11"
        assert not np.any(R & ~(used | (used << np.uint64(1)))), "bits set outside the entries"
        w0 = R[:, 0]
        assert not np.any((w0 >> np.uint64(1)) & ~w0 & ubox), "negative box entry"
        for k in range(D):
            at_lo = ((w0 >> np.uint64(4 * k)) & np.uint64(3)) == 0
            at_hi = ((w0 >> np.uint64(4 * k + 2)) & np.uint64(3)) == 0
            assert np.all(x[at_lo, k] == box.lo[k]) and np.all(x[at_hi, k] == box.hi[k]), "box coordinate"
            inner = ~(at_lo | at_hi)
            assert np.all((x[inner, k] > box.lo[k]) & (x[inner, k] < box.hi[k])), "vertex outside the box"
        nzb = (w0 | (w0 >> np.uint64(1))) & MASK01
        zbox[s0:s0 + chunk] = np.bitwise_count(ubox & ~nzb)
        keys[s0:s0 + chunk] = (R * mult).sum(axis=1, dtype=np.uint64)
    # distinct rows: rows whose keys collide are compared exactly
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    eq = ks[1:] == ks[:-1]
    in_group = np.zeros(info.V, bool)
    in_group[:-1] |= eq
    in_group[1:] |= eq
    rows = SG[order[in_group]]
    print(f"[full] {len(rows)} rows share a key with another row; compared exactly", flush=True)
    assert len(np.unique(rows, axis=0)) == len(rows), "duplicate sign-vectors"
    deg = np.bincount(Ed.ravel(), minlength=info.V)
    assert len(deg) == info.V, "edge endpoint out of range"
    assert np.array_equal(deg, 2 * D - zbox), "degree != 2D - z_box"
    assert 2 * info.E == int((2 * D - zbox).sum())


def test_full_sampled_edges(full):
    net, box, info, steps, X, SG, Ed = full
    D = 3
    used, _ = _word_masks(net.widths)
    rng = np.random.default_rng(11)
    idx = rng.choice(info.E, 1 << 21, replace=False)
    a, b = Ed[idx, 0].astype(np.int64), Ed[idx, 1].astype(np.int64)
    assert np.all(a != b)
    Ra, Rb = SG[a], SG[b]
    za = ~((Ra | (Ra >> np.uint64(1))) & MASK01)
    zb = ~((Rb | (Rb >> np.uint64(1))) & MASK01)
    shared = np.bitwise_count(used & za & zb).sum(axis=1)
    assert np.all(shared == D - 1), "edge without D-1 shared zeros"
    pa, na = Ra & ~(Ra >> np.uint64(1)) & MASK01, (Ra >> np.uint64(1)) & ~Ra & MASK01
    pb, nb = Rb & ~(Rb >> np.uint64(1)) & MASK01, (Rb >> np.uint64(1)) & ~Rb & MASK01
    assert not np.any((pa & nb) | (na & pb)), "edge endpoints in conflict"
    # midpoints of a smaller sample lie in the edge's cell (all 774 entries)
    sub = slice(0, 4096)
    Sa = unpack_signs(Ra[sub], net.widths)
    Sb = unpack_signs(Rb[sub], net.widths)
    jn = np.where(Sa == 0, Sb, Sa)
    mid = 0.5 * (X[a[sub]] + X[b[sub]])
    mv = brute.entry_values(net, box.lo, box.hi, mid)
    assert np.all(np.abs(mv[jn == 0]) < 1e-7), "edge leaves a hyperplane it should lie on"
    assert np.all(np.sign(mv[jn != 0]) == jn[jn != 0]), "edge midpoint outside its cell"


def test_full_sampled_vertices(oracle_lib, full):
    net, box, info, steps, X, SG, Ed = full
    rng = np.random.default_rng(12)
    idx = np.sort(rng.choice(info.V, 4096, replace=False))
    S = unpack_signs(SG[idx], net.widths)
    x = oracle_lib.vertex_solve(net, box.lo, box.hi, S)
    err = np.abs(x - X[idx]).max()
    print(f"[full] sampled vertices: max |x_solve - x_gpu| = {err:.3g}", flush=True)
    assert err < 1e-9
    z = oracle_lib.forward(net, X[idx])[:, :768]
    Sn = S[:, 6:]
    assert np.all(np.abs(z[Sn == 0]) < 1e-9), f"max |z| at zeros {np.abs(z[Sn == 0]).max()}"
    assert np.all(np.sign(z[Sn != 0]) == Sn[Sn != 0]), "forward-pass sign differs from the sign-vector"


def test_large_net_small_box_matches_oracle(oracle_lib, pcx):
    """The same network on a small centred box, compared whole with the oracle
    (every layer subdivided)."""
    net = wl.plain_large()
    lo, hi = np.full(3, -0.05), np.full(3, 0.05)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, lo, hi)
    X, SG, Ed = cx.copy()
    steps = cx.steps()
    cx.close()
    m.close()
    S = unpack_signs(SG, net.widths)
    r = oracle_lib.extract(net, lo, hi)
    assert np.array_equal(steps, r.steps)
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)
    check_invariants(net, lo, hi, X, S, Ed, full=False)


@pytest.mark.timeout(900)
def test_large_net_subbox_whole_on_full_grids(oracle_lib, pcx, monkeypatch):
    """The same network on the centred box [-0.125, 0.125]^3 (1.0M vertices,
    3.0M edges, up to 17K splits and 68K 2-face key slots in a step), every
    layer subdivided, compared whole with the oracle. The extraction runs twice:
    with the launch shapes chosen for these step sizes, and with every step's
    compaction, split and pairing on their largest grids (1024 compaction and
    pairing workgroups, 16384 split workgroups: the shape of the bench's big
    steps); both give the same arrays."""
    from conftest import oracle_pool, oracle_threads
    net = wl.plain_large()
    lo, hi = np.full(3, -0.125), np.full(3, 0.125)
    pool = oracle_pool()
    fut = pool.submit(oracle_lib.extract, net, lo, hi, False, 0, False, oracle_threads())
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, lo, hi)
    base = cx.copy()
    cx.close()
    monkeypatch.setenv("PCX_FULL_GRIDS", "1")
    cx = pcx.extract(m, lo, hi)
    X, SG, Ed = cx.copy()
    steps = cx.steps()
    cx.close()
    monkeypatch.delenv("PCX_FULL_GRIDS")
    m.close()
    for a, b in zip((X, SG, Ed), base):
        assert a.shape == b.shape and np.array_equal(a, b), "launch shape changed the result"
    print(f"[subbox] V={len(X)} E={len(Ed)} largest step {steps[:, 2].max()} splits, "
          f"{steps[:, 3].max()} key slots", flush=True)
    r = fut.result()
    pool.shutdown()
    assert len(Ed) >= 2_000_000
    assert np.array_equal(steps, r.steps)
    S = unpack_signs(SG, net.widths)
    del SG, base
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)
