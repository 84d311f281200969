"""Seeded synthetic inputs: random ReLU MLPs and input boxes.

This module only draws numbers. It holds none of the extraction arithmetic, so
the GPU library and the CPU oracle can both be fed from it without sharing any
part of the method.

Networks follow the paper's experimental setting (Sec. 5.1.2: randomly
initialised fully connected ReLU networks on a hypercube domain) with the
layer definition x^(l) = ReLU(W^(l) x^(l-1) + b^(l)) of Sec. 3.4:

* ``W^(l)`` has shape ``[N_l, N_{l-1}]`` (torch ``Linear`` layout, z = W x + b),
  drawn He-normal: ``standard_normal * sqrt(2 / N_{l-1})``;
* ``b^(l)`` is drawn ``uniform(-0.5, 0.5)``;
* draw order is W1, b1, W2, b2, ..., from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np


@dataclass
class Net:
    """A ReLU MLP: ``widths = [D, N_1, ..., N_{L-1}, N_out]``."""

    widths: List[int]
    W: List[np.ndarray]
    b: List[np.ndarray]
    name: str = ""

    @property
    def D(self) -> int:
        return self.widths[0]


@dataclass
class Box:
    lo: np.ndarray
    hi: np.ndarray


def he_mlp(widths: Sequence[int], seed, name: str = "") -> Net:
    """He-normal weights, U(-0.5, 0.5) biases, drawn W1, b1, W2, b2, ..."""
    rng = np.random.default_rng(seed)
    W, b = [], []
    for l in range(1, len(widths)):
        fan_in, fan_out = int(widths[l - 1]), int(widths[l])
        W.append(np.ascontiguousarray(
            rng.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in), dtype=np.float64))
        b.append(np.ascontiguousarray(rng.uniform(-0.5, 0.5, fan_out), dtype=np.float64))
    return Net([int(w) for w in widths], W, b, name)


def cube(D: int, half: float = 1.0) -> Box:
    return Box(np.full(D, -half, dtype=np.float64), np.full(D, half, dtype=np.float64))


# --- the five workloads -----------------------------------------------------

def plain_small() -> Net:
    """2 -> 8 -> 8 -> 1 on [-1,1]^2, seed 1."""
    return he_mlp([2, 8, 8, 1], 1, "mlp-2-8-8-1")


def plain_large() -> Net:
    """3 -> 256 -> 256 -> 256 -> 1 on [-1,1]^3, seed 2 (768 hidden neurons)."""
    return he_mlp([3, 256, 256, 256, 1], 2, "mlp-3-256x3-1")


def batch_archs(n: int = 4096, seed: int = 3):
    """Architectures 2 -> [w] x d -> 1, w in {8,16,32,64}, d in {2,3,4}."""
    rng = np.random.default_rng(seed)
    ws = rng.choice([8, 16, 32, 64], size=n)
    ds = rng.choice([2, 3, 4], size=n)
    return [[2] + [int(w)] * int(d) + [1] for w, d in zip(ws, ds)]


def batch_nets(n: int = 4096, seed: int = 3) -> List[Net]:
    archs = batch_archs(n, seed)
    return [he_mlp(a, [seed, i], f"batch-{i}") for i, a in enumerate(archs)]


@dataclass
class Request:
    net: Net
    box: Box
    arrival_s: float


def serve_requests(n: int = 2000, rate_per_s: float = 1000.0, seed: int = 4) -> List[Request]:
    """Poisson arrivals; D in {2,3}, constant width in [16,128], depth in {2,3,4}."""
    rng = np.random.default_rng(seed)
    Ds = rng.choice([2, 3], size=n)
    widths = rng.integers(16, 129, size=n)
    depths = rng.choice([2, 3, 4], size=n)
    gaps = rng.exponential(1.0, size=n)  # unit-rate gaps, scaled below
    t = np.cumsum(gaps) / float(rate_per_s)
    out = []
    for i in range(n):
        arch = [int(Ds[i])] + [int(widths[i])] * int(depths[i]) + [1]
        out.append(Request(he_mlp(arch, [seed, i], f"req-{i}"), cube(int(Ds[i])), float(t[i])))
    return out


def differentiable() -> Net:
    """3 -> 64 -> 64 -> 64 -> 1 on [-1,1]^3, seed 5 (output neuron subdivided too)."""
    return he_mlp([3, 64, 64, 64, 1], 5, "mlp-3-64x3-1")


def differentiable_small() -> Net:
    """3 -> 8 -> 8 -> 1 sibling of the differentiable workload (cheap finite differences)."""
    return he_mlp([3, 8, 8, 1], 5, "mlp-3-8-8-1")
