"""torch.autograd.Function over the C ABI: vertex coordinates of the extracted
complex as a differentiable function of the weights and biases.

PyTorch provides device memory and the stream only: the extraction runs in
``pcx_extract`` and the gradient in the hand-written backward kernels behind
``pcx_backward`` (the reverse of the interpolation x0 = x_p + t (x_q - x_p),
t = z_p / (z_p - z_q), Sec. 4.2.1 of the paper).
"""
from __future__ import annotations

from typing import List, Sequence

import torch

from . import pcx


def _stream():
    return torch.cuda.current_stream().cuda_stream


class ExtractCoords(torch.autograd.Function):
    """forward(lo, hi, precision, include_output, W1, b1, ..., WL, bL) ->
    (coords [V, D] float64, signs [V, Wd] int64 (raw 64-bit words), edges [E, 2] int32).
    Only coords is differentiable."""

    @staticmethod
    def forward(ctx, lo, hi, precision, include_output, *params):
        Ws, bs = params[0::2], params[1::2]
        widths = [int(Ws[0].shape[1])] + [int(W.shape[0]) for W in Ws]
        mlp = pcx.MLP(widths, [W.detach().cpu().double().numpy() for W in Ws],
                      [b.detach().cpu().double().numpy() for b in bs])
        cx = pcx.extract(mlp, lo.detach().cpu().double().numpy(), hi.detach().cpu().double().numpy(),
                         include_output=bool(include_output), record_tape=True, stream=_stream())
        info = cx.info()
        dev = Ws[0].device
        X = torch.empty((info.V, info.D), dtype=torch.float64, device=dev)
        SG = torch.empty((info.V, info.Wd), dtype=torch.int64, device=dev)
        Ed = torch.empty((info.E, 2), dtype=torch.int32, device=dev)
        cx.copy_device(X.data_ptr(), SG.data_ptr(), Ed.data_ptr(), _stream())
        ctx.mlp, ctx.cx, ctx.precision = mlp, cx, int(precision)
        ctx.shapes = [(W.shape, b.shape) for W, b in zip(Ws, bs)]
        ctx.mark_non_differentiable(SG, Ed)
        return X, SG, Ed

    @staticmethod
    def backward(ctx, gX, gSG, gEd):
        dev = gX.device
        g = gX.contiguous().to(torch.float64)
        gW = [torch.empty(ws, dtype=torch.float64, device=dev) for ws, _ in ctx.shapes]
        gb = [torch.empty(bs, dtype=torch.float64, device=dev) for _, bs in ctx.shapes]
        pcx.backward(ctx.mlp, ctx.cx, g.data_ptr(), [t.data_ptr() for t in gW], [t.data_ptr() for t in gb],
                     ctx.precision, _stream())
        grads = []
        for a, c in zip(gW, gb):
            grads += [a, c]
        return (None, None, None, None, *grads)


def extract_coords(Ws: Sequence[torch.Tensor], bs: Sequence[torch.Tensor], lo, hi, include_output=True,
                   precision: str = "f64"):
    """Coordinates (differentiable), packed signs and edges of the complex."""
    params: List[torch.Tensor] = []
    for W, b in zip(Ws, bs):
        params += [W, b]
    prec = pcx.PCX_F64 if precision == "f64" else pcx.PCX_F32
    lo = torch.as_tensor(lo, dtype=torch.float64)
    hi = torch.as_tensor(hi, dtype=torch.float64)
    return ExtractCoords.apply(lo, hi, prec, bool(include_output), *params)


def level_set_mask(signs: torch.Tensor, widths: Sequence[int], include_output=True) -> torch.Tensor:
    """Vertices whose output entry (the first output neuron) is 0."""
    assert include_output
    lw = 1
    for n in widths[1:-1]:
        lw += (int(n) + 31) // 32
    return (signs[:, lw] & 3) == 0


def level_set_edge_loss(X: torch.Tensor, signs: torch.Tensor, edges: torch.Tensor, widths) -> torch.Tensor:
    """Sum of squared lengths of the edges on the zero level set of the output
    (both endpoints carry 0 at the output entry)."""
    on = level_set_mask(signs, widths)
    e = edges.long()
    keep = on[e[:, 0]] & on[e[:, 1]]
    d = X[e[keep, 0]] - X[e[keep, 1]]
    return (d * d).sum()
