"""GPU parity on a simplex domain (pcx_extract_simplex): bit-exact sign-vectors,
per-step counters and canonical incidence against the oracle, coordinates
within 1e-10; with the output level set, pruning and both pairing modes."""
import numpy as np
import pytest

from checks import assert_same_complex, level_set, unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu

S2 = np.array([[-1.0, -1.0], [1.5, -0.8], [-0.7, 1.3]])
S3 = np.array([[-1.0, -1, -1], [1.2, -0.9, -1.1], [-0.8, 1.4, -0.7], [-0.9, -0.6, 1.5]])
S1 = np.array([[-1.0], [1.0]])


def _simplex(D, seed):
    """A random simplex around the origin: D + 1 corners in general position."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.5, 1.5, (D + 1, D))


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def run(pcx, net, corners, **kw):
    m = pcx.MLP.from_net(net)
    cx = pcx.extract_simplex(m, corners, **kw)
    X, SG, Ed = cx.copy()
    S = unpack_signs(SG, net.widths, kw.get("include_output", False), m=net.D + 1)
    steps = cx.steps()
    cx.close()
    m.close()
    return X, S, Ed, steps


CASES = [([2, 5, 4, 1], 3, S2, False), ([2, 16, 16, 1], 41, S2, False), ([3, 4, 3, 1], 7, S3, False),
         ([3, 24, 20, 1], 42, S3, False), ([3, 12, 12, 1], 43, S3, True), ([4, 8, 8, 1], 44, None, False),
         ([1, 7, 7, 1], 45, S1, False), ([5, 6, 6, 1], 46, None, True)]


@pytest.mark.parametrize("widths,seed,corners,incl", CASES)
@pytest.mark.parametrize("pairing", ["hash", "sort"])
def test_simplex_matches_oracle(oracle_lib, pcx, widths, seed, corners, incl, pairing):
    net = wl.he_mlp(widths, seed)
    P = _simplex(widths[0], seed) if corners is None else corners
    X, S, Ed, steps = run(pcx, net, P, include_output=incl, pairing=pairing)
    r = oracle_lib.extract_simplex(net, P, include_output=incl)
    assert np.array_equal(steps, r.steps), "per-step counters differ"
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)
    D = widths[0]
    zdom = (S[:, :D + 1] == 0).sum(1)
    assert np.array_equal(np.bincount(Ed.ravel(), minlength=len(X)), 2 * D - zdom)


def test_simplex_pruned_level_set(oracle_lib, pcx):
    net = wl.he_mlp([3, 16, 16, 16, 1], 55)  # level set of 242 vertices; 528 of 2727 vertices survive
    X, S, Ed, steps = run(pcx, net, S3, include_output=True, prune=True)
    r = oracle_lib.extract_simplex(net, S3, include_output=True, prune=True)
    assert np.array_equal(steps, r.steps)
    assert_same_complex((X, S, Ed), (r.X, r.S, r.edges), coord_tol=1e-10)
    Xf, Sf, Ef, _ = run(pcx, net, S3, include_output=True)
    assert_same_complex(level_set(X, S, Ed), level_set(Xf, Sf, Ef), coord_tol=0.0)


def test_degenerate_simplex_is_rejected(pcx):
    net = wl.he_mlp([2, 4, 1], 3)
    m = pcx.MLP.from_net(net)
    flat = np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 2.0]])
    with pytest.raises(pcx.PcxError) as e:
        pcx.extract_simplex(m, flat)
    assert e.value.code == pcx.PCX_ERR_INVALID
    m.close()
