"""GPU backward (pcx_backward via torch.autograd.Function) against references
that never touch the HIP path: central differences of the oracle's loss, and
the implicit-function closed form evaluated on the oracle's complex.

Loss: sum of squared lengths of the edges on the zero level set of the output.
"""
import numpy as np
import pytest

from implicit import implicit_grad, level_set_loss, oracle_fd
from paper_2306_07212_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_ops():
    import torch
    assert torch.cuda.is_available()
    from paper_2306_07212_amd import torch_ops as T
    return T


def gpu_grads(torch_ops, net, precision="f64"):
    import torch
    dev = torch.device("cuda:0")
    Ws = [torch.tensor(w, dtype=torch.float64, device=dev, requires_grad=True) for w in net.W]
    bs = [torch.tensor(x, dtype=torch.float64, device=dev, requires_grad=True) for x in net.b]
    box = wl.cube(net.D)
    X, SG, Ed = torch_ops.extract_coords(Ws, bs, box.lo, box.hi, include_output=True, precision=precision)
    loss = torch_ops.level_set_edge_loss(X, SG, Ed, net.widths)
    loss.backward()
    return (float(loss.item()), [w.grad.cpu().numpy() for w in Ws], [b.grad.cpu().numpy() for b in bs], len(X))


def rel(a, b):
    num = sum(np.sum((x - y) ** 2) for x, y in zip(a, b))
    den = sum(np.sum(y ** 2) for y in b)
    return float(np.sqrt(num / den))


def test_backward_matches_oracle_finite_differences(oracle_lib, torch_ops):
    net = wl.differentiable_small()
    box = wl.cube(3)
    loss, gW, gb, V = gpu_grads(torch_ops, net)
    r = oracle_lib.extract(net, box.lo, box.hi, include_output=True)
    L, _, _ = level_set_loss(r.X, r.S, r.edges, net.widths)
    assert V == r.V
    assert abs(loss - L) <= 1e-12 * max(1.0, abs(L))
    fW, fb = oracle_fd(oracle_lib, net, box)
    assert rel(gW + gb, fW + fb) < 1e-6


def test_backward_matches_implicit_closed_form_full_workload(oracle_lib, torch_ops):
    """3 -> 64 -> 64 -> 64 -> 1, level set of the output: 0.67M vertices."""
    net = wl.differentiable()
    box = wl.cube(3)
    loss, gW, gb, V = gpu_grads(torch_ops, net)
    r = oracle_lib.extract(net, box.lo, box.hi, include_output=True)
    L, G, nedges = level_set_loss(r.X, r.S, r.edges, net.widths)
    assert V == r.V and nedges > 1000
    assert abs(loss - L) <= 1e-9 * abs(L)
    iW, ib = implicit_grad(net, box.lo, box.hi, r.X, r.S, G)
    assert rel(gW + gb, iW + ib) < 1e-8


def test_fp32_backward_error(torch_ops):
    """FP32 reverse pass on the FP64 forward: relative error against FP64."""
    net = wl.differentiable()
    _, gW, gb, _ = gpu_grads(torch_ops, net, "f64")
    _, fW, fb, _ = gpu_grads(torch_ops, net, "f32")
    err = rel(fW + fb, gW + gb)
    print(f"fp32 backward relative error vs fp64: {err:.3e}")
    assert err < 1e-4


def test_backward_needs_the_tape():
    from paper_2306_07212_amd import pcx
    net = wl.differentiable_small()
    box = wl.cube(3)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi, include_output=True)
    with pytest.raises(pcx.PcxError) as e:
        pcx.backward(m, cx, 1, [1] * 3, [1] * 3)
    assert e.value.code == pcx.PCX_ERR_INVALID


def test_backward_is_deterministic():
    """Repeated backward passes over the same tape and the same dL/dx give the
    same gradient bits, in FP64 and in FP32: each parent sums its children's
    contributions in child order, with no atomic accumulation."""
    import torch
    from paper_2306_07212_amd import pcx
    net = wl.differentiable()
    box = wl.cube(3)
    m = pcx.MLP.from_net(net)
    cx = pcx.extract(m, box.lo, box.hi, include_output=True, record_tape=True)
    V = cx.info().V
    dev = torch.device("cuda:0")
    g = torch.tensor(np.random.default_rng(9).standard_normal((V, 3)), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    for prec in (pcx.PCX_F64, pcx.PCX_F32):
        runs = []
        for _ in range(3):
            gW = [torch.full(w.shape, np.nan, dtype=torch.float64, device=dev) for w in net.W]
            gb = [torch.full(b.shape, np.nan, dtype=torch.float64, device=dev) for b in net.b]
            pcx.backward(m, cx, g.data_ptr(), [t.data_ptr() for t in gW], [t.data_ptr() for t in gb], prec, stream)
            torch.cuda.synchronize()
            runs.append([t.cpu().numpy() for t in gW + gb])
        for r in runs[1:]:
            for a, b in zip(r, runs[0]):
                assert np.all(np.isfinite(a)) and np.array_equal(a, b), "gradients differ between runs"
    cx.close()
    m.close()
