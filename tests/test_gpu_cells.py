"""GPU cell reconstruction (pcx_cell_counts, pcx_regions) against the oracle's
plain perturbation: f-vectors equal, region sign-vectors equal as sets; on the
768-neuron workload the alternating sum of the f-vector is 1 (Euler)."""
import numpy as np
import pytest

from checks import unpack_signs
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu

S2 = np.array([[-1.0, -1.0], [1.5, -0.8], [-0.7, 1.3]])
S3 = np.array([[-1.0, -1, -1], [1.2, -0.9, -1.1], [-0.8, 1.4, -0.7], [-0.9, -0.6, 1.5]])

CASES = [([2, 8, 8, 1], 1, None, False), ([3, 8, 8, 1], 5, None, False), ([3, 10, 10, 10, 1], 32, None, False),
         ([4, 6, 6, 1], 34, None, False), ([1, 6, 6, 1], 33, None, False), ([2, 5, 4, 1], 3, S2, False),
         ([3, 4, 3, 1], 7, S3, False), ([3, 8, 8, 1], 5, None, True), ([2, 40, 40, 1], 51, None, False),
         ([5, 5, 5, 1], 52, None, False)]


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


@pytest.mark.parametrize("widths,seed,P,incl", CASES)
def test_cells_match_oracle(oracle_lib, pcx, widths, seed, P, incl):
    from oracle.cells import face_counts
    net = wl.he_mlp(widths, seed)
    D = widths[0]
    m = pcx.MLP.from_net(net)
    if P is None:
        box = wl.cube(D)
        cx = pcx.extract(m, box.lo, box.hi, include_output=incl)
        r = oracle_lib.extract(net, box.lo, box.hi, include_output=incl)
        mdom = 2 * D
    else:
        cx = pcx.extract_simplex(m, P, include_output=incl)
        r = oracle_lib.extract_simplex(net, P, include_output=incl)
        mdom = D + 1
    f = cx.cell_counts()
    rows = cx.regions()
    cx.close()
    m.close()
    fo, regs = face_counts(r.S, r.edges, D, mdom)
    assert list(f) == list(fo)
    assert sum((-1) ** k * int(x) for k, x in enumerate(f)) == 1
    S = unpack_signs(rows, widths, incl, m=mdom)
    assert len(S) == len(regs)
    assert {row.tobytes() for row in S} == {row.tobytes() for row in regs}
    # sorted rows, no zeros left
    assert not np.any(S == 0)
    assert all(tuple(a) <= tuple(b) for a, b in zip(rows[:-1], rows[1:]))


def test_cells_of_the_768_neuron_workload(pcx):
    """3.8e7 vertices: f = (V, E, F, C) with V - E + F - C = 1."""
    net = wl.plain_large()
    box = wl.cube(3)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi)
    f = cx.cell_counts()
    print(f"[cells] f-vector {list(map(int, f))}", flush=True)
    cx.close()
    m.close()
    assert f[0] == 37675286 and f[1] == 112775239
    assert int(f[0]) - int(f[1]) + int(f[2]) - int(f[3]) == 1
