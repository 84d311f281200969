"""pcx_extract_into: the extraction written into caller-allocated device
buffers, every other array in the library's static scratch (no device
allocation by the library). Its complexes must equal pcx_extract's (the same
arrays, numbering and per-step counters), on consecutive calls whose second is
smaller than the first (the scratch keeps the first call's contents)."""
import numpy as np
import pytest

from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcx():
    from paper_2306_07212_amd import pcx as P
    return P


def reference(pcx, net, incl):
    m = pcx.MLP.from_net(net)
    box = wl.cube(net.D)
    cx = pcx.extract(m, box.lo, box.hi, include_output=incl)
    out = cx.copy()
    steps = cx.steps()
    info = cx.info()
    cx.close()
    m.close()
    return out, steps, info


def into(pcx, net, incl, max_v, max_e):
    import torch
    dev = torch.device("cuda:0")
    L = len(net.widths) - 1
    wd = 1 + sum((w + 31) // 32 for w in net.widths[1:L + 1 if incl else L])
    X = torch.full((max_v, net.D), np.nan, dtype=torch.float64, device=dev)
    SG = torch.full((max_v, wd), -1, dtype=torch.int64, device=dev)
    Ed = torch.full((max_e, 2), -7, dtype=torch.int32, device=dev)
    m = pcx.MLP.from_net(net)
    box = wl.cube(net.D)
    info, steps = pcx.extract_into(m, box.lo, box.hi, X.data_ptr(), SG.data_ptr(), Ed.data_ptr(), max_v, max_e,
                                   include_output=incl, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    m.close()
    out = (X[:info.V].cpu().numpy(), SG[:info.V].cpu().numpy().view(np.uint64), Ed[:info.E].cpu().numpy())
    return out, steps, info


def test_two_calls_in_a_row_match_pcx_extract(pcx):
    # a larger complex first, then a smaller one on the same scratch
    for net, incl in [(wl.he_mlp([3, 24, 24, 1], 71), True), (wl.plain_small(), False)]:
        ref, rsteps, rinfo = reference(pcx, net, incl)
        got, steps, info = into(pcx, net, incl, max_v=4 * rinfo.V + 64, max_e=4 * rinfo.E + 64)
        print(f"[into] {net.widths}: V={info.V} E={info.E} scratch={info.peak_bytes} B", flush=True)
        assert (info.V, info.E, info.total_splits, info.total_pairs) == (rinfo.V, rinfo.E, rinfo.total_splits,
                                                                         rinfo.total_pairs)
        assert np.array_equal(steps, rsteps)
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b), "pcx_extract_into differs from pcx_extract"


def test_capacity_errors_are_reported(pcx):
    net = wl.plain_small()
    ref, _, rinfo = reference(pcx, net, False)
    with pytest.raises(pcx.PcxError) as e:
        into(pcx, net, False, max_v=rinfo.V - 1, max_e=4 * rinfo.E)
    assert e.value.code == pcx.PCX_ERR_CAPACITY
    # maxima whose scratch would not fit are refused before any work
    with pytest.raises(pcx.PcxError) as e:
        into(pcx, wl.plain_large(), False, max_v=1 << 22, max_e=1 << 23)
    assert e.value.code == pcx.PCX_ERR_CAPACITY and "scratch" in str(e.value)
    # maxima near 2^31 (key slots beyond 32 bits) are refused the same way, before any buffer is touched
    import torch
    dev = torch.device("cuda:0")
    tiny = [torch.zeros(8, dtype=t, device=dev) for t in (torch.float64, torch.int64, torch.int32)]
    m = pcx.MLP.from_net(wl.plain_large())
    box = wl.cube(3)
    with pytest.raises(pcx.PcxError) as e:
        pcx.extract_into(m, box.lo, box.hi, tiny[0].data_ptr(), tiny[1].data_ptr(), tiny[2].data_ptr(),
                         (1 << 31) - 2, (1 << 31) - 2)
    assert e.value.code == pcx.PCX_ERR_CAPACITY and "scratch" in str(e.value)
    m.close()
    # and the entry point still works after all of them
    got, _, info = into(pcx, net, False, max_v=4 * rinfo.V, max_e=4 * rinfo.E)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
