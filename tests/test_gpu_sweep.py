"""A seeded sweep over network shapes: input dimensions 1 to 8, one to three
hidden layers of widths 1 to 140, with and without the output level set. Every
network is extracted in one batched launch (under the default and the 32-lane
schedules) and on the per-step kernels; the three must agree bit for bit
(values, numbering, per-step counters) and with the oracle's complex in
canonical form. The shapes cross every split-group width (16 and 32 lanes),
the evaluation kernels (MFMA strips, the LDS tile, the one-vertex-per-thread
and register-tiled kernels) and key counts from 0 (D = 1) to 14 (D = 8)."""
import numpy as np
import pytest

from checks import assert_same_complex, unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu


def shapes(n=48, seed=20261203):
    """Seeded shapes whose complexes stay small enough for the oracle (the
    subdivided neurons bounded per input dimension)."""
    rng = np.random.default_rng(seed)
    budget = {1: 300, 2: 220, 3: 60, 4: 24, 5: 14, 6: 11, 7: 9, 8: 8}
    out = []
    while len(out) < n:
        D = int(rng.integers(1, 9))
        depth = int(rng.integers(1, 4))
        cap = budget[D]
        widths = [int(rng.integers(1, max(2, min(140, cap // depth) + 1))) for _ in range(depth)]
        if sum(widths) > cap:
            continue
        incl = bool(rng.integers(0, 2))
        out.append(([D] + widths + [1], incl))
    return out


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


@pytest.mark.parametrize("incl", [False, True])
def test_shape_sweep_batched_per_step_and_oracle(pcx, oracle_lib, monkeypatch, incl):
    monkeypatch.setenv("PCX_NO_TINY", "1")   # the per-step reference runs the per-step kernels
    monkeypatch.setenv("PCX_NO_GRAPH", "1")
    arch = [(w, i) for w, i in shapes() if i == incl]
    nets = [wl.he_mlp(w, [77, k]) for k, (w, _) in enumerate(arch)]
    mlps = [pcx.MLP.from_net(n) for n in nets]
    boxes = [(wl.cube(n.D).lo, wl.cube(n.D).hi) for n in nets]
    runs = {}
    for sched in ("4", "0"):   # 16 lanes per split (the default), 32 lanes
        monkeypatch.setenv("PCX_BATCH_SCHED", sched)
        bt = pcx.Batch(mlps, boxes, include_output=incl)
        st = bt.stats()
        print(f"[sweep] incl={incl} schedule {sched}: {st.n} networks, {st.total_V} vertices, "
              f"{st.fallbacks} on the per-step path", flush=True)
        runs[sched] = [(bt.copy(i), bt.steps(i)) for i in range(len(nets))]
        bt.close()
    for i, net in enumerate(nets):
        box = wl.cube(net.D)
        cx = pcx.extract(mlps[i], box.lo, box.hi, include_output=incl)
        ref, rsteps = cx.copy(), cx.steps()
        cx.close()
        for sched, got in runs.items():
            (arrs, steps) = got[i]
            for a, b in zip(arrs, ref):
                assert a.shape == b.shape and np.array_equal(a, b), f"{net.widths} schedule {sched}"
            assert np.array_equal(steps, rsteps), f"{net.widths} schedule {sched}: per-step counters"
        r = oracle_lib.extract(net, box.lo, box.hi, include_output=incl)
        X, SG, Ed = ref
        assert np.array_equal(rsteps, r.steps), f"{net.widths}: per-step counters vs the oracle"
        assert_same_complex((X, unpack_signs(SG, net.widths, incl), Ed), (r.X, r.S, r.edges))
    for m in mlps:
        m.close()
