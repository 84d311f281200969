"""GPU parity of pruning during subdivision (Sec. 5.4.2, pcx_opts.prune).

The pruned complex (after every layer start's pruning, then the output neuron's
subdivision) equals the oracle's pruned complex: bit-exact sign-vectors,
per-step counters and canonical incidence, coordinates within 1e-10. Its level
set equals the unpruned GPU extraction's level set point for point.
"""
import numpy as np
import pytest

from checks import assert_same_complex, level_set, unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASES = [([2, 8, 8, 1], 1), ([3, 8, 8, 1], 5), ([2, 16, 16, 16, 1], 7), ([2, 12, 10, 1], 31),
         ([3, 10, 10, 10, 1], 32), ([1, 6, 6, 1], 33), ([4, 6, 6, 1], 34), ([3, 40, 150, 1], 35)]


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def run(pcx, net, box, **kw):
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi, include_output=True, **kw)
    X, SG, Ed = cx.copy()
    S = unpack_signs(SG, net.widths, True)
    steps = cx.steps()
    cx.close()
    m.close()
    return X, S, Ed, steps


@pytest.mark.parametrize("widths,seed", CASES)
@pytest.mark.parametrize("pairing", ["hash", "sort"])
def test_pruned_matches_oracle(oracle_lib, pcx, widths, seed, pairing):
    net = wl.he_mlp(widths, seed)
    box = wl.cube(widths[0])
    X, S, Ed, steps = run(pcx, net, box, prune=True, pairing=pairing)
    r = oracle_lib.extract(net, box.lo, box.hi, include_output=True, prune=True)
    assert np.array_equal(steps, r.steps), "per-step counters differ"
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)
    # the level set is untouched by pruning
    Xf, Sf, Ef, _ = run(pcx, net, box, pairing=pairing)
    assert_same_complex(level_set(X, S, Ed), level_set(Xf, Sf, Ef), coord_tol=0.0)


def test_pruned_level_set_of_the_differentiable_workload(oracle_lib, pcx):
    """3-64-64-64-1 with the output: 26.5K vertices pruned vs 670K in full."""
    net = wl.differentiable()
    box = wl.cube(3)
    X, S, Ed, steps = run(pcx, net, box, prune=True)
    r = oracle_lib.extract(net, box.lo, box.hi, include_output=True, prune=True)
    assert np.array_equal(steps, r.steps)
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)
    Xf, Sf, Ef, _ = run(pcx, net, box)
    assert len(Xf) == 670310
    assert_same_complex(level_set(X, S, Ed), level_set(Xf, Sf, Ef), coord_tol=0.0)


def test_prune_argument_errors(pcx):
    net = wl.he_mlp([2, 4, 1], 3)
    box = wl.cube(2)
    m = pcx.MLP.from_net(net)
    with pytest.raises(pcx.PcxError) as e:
        pcx.extract(m, box.lo, box.hi, include_output=False, prune=True)
    assert e.value.code == pcx.PCX_ERR_INVALID
    with pytest.raises(pcx.PcxError) as e:
        pcx.extract(m, box.lo, box.hi, include_output=True, prune=True, record_tape=True)
    assert e.value.code == pcx.PCX_ERR_INVALID
    cx = pcx.extract(m, box.lo, box.hi, include_output=True, prune=True)
    with pytest.raises(pcx.PcxError) as e:
        cx.cell_counts()
    assert e.value.code == pcx.PCX_ERR_INVALID
    cx.close()
    m.close()
