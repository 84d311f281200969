#!/usr/bin/env python3
"""Benchmark of edge-subdivision polyhedral complex extraction on one MI355X.

One step = one full extraction (``pcx_extract``) of the 1-skeleton of the
3 -> 256 -> 256 -> 256 -> 1 ReLU MLP (He-normal weights, U(-0.5, 0.5) biases,
seed 2) on the box [-1, 1]^3: all 768 hidden neurons, weights resident in HBM
before the timed region, the complex resident in HBM after it.

Prints one JSON line. ``value`` is edges subdivided per second (splitting
edges summed over all neuron steps / wall time per extraction); vertices/s and
edges/s of the final complex are reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 (vector and matrix)
METRIC = "edges subdivided/s + vertices/s (plain vs batched/served), p50/p99 extraction latency"
FAMILIES = ["gemm", "next", "select", "split", "sort", "pair"]


def layer_table(widths, include_output=False):
    D = widths[0]
    L = len(widths) - 1
    nsub = L if include_output else L - 1
    lw = 1
    out = []
    for l in range(1, nsub + 1):
        N = widths[l]
        nw = (N + 31) // 32
        out.append(dict(K=widths[l - 1], N=N, lw0=lw, nw=nw))
        lw += nw
    return out, lw


def algorithmic_cost(widths, steps, include_output=False):
    """Bytes (and FLOPs for the evaluation) each kernel family must move for the
    work of one extraction; the per-unit figures are stated in the design doc."""
    D = widths[0]
    layers, Wd = layer_table(widths, include_output)
    ZS = max(x["N"] for x in layers)
    P = 2 * (D - 1)
    by = dict.fromkeys(FAMILIES, 0.0)
    flops = 0.0
    s0 = 0
    for ly in layers:
        N, K, nw = ly["N"], ly["K"], ly["nw"]
        V0, E0 = steps[s0, 0], steps[s0, 1]
        kin = D if s0 == 0 else K
        flops += 2.0 * V0 * kin * N
        by["gemm"] += V0 * (8.0 * kin + 8.0 * N + 8.0 * nw)
        by["next"] += E0 * (8.0 + 2 * 8.0 * nw + 2.0)
        for j, st in enumerate(steps[s0:s0 + N]):
            V, E, S, Kv = (float(v) for v in st)
            wn = ly["lw0"] + j // 32  # face sign-vectors span words 0..wn
            by["select"] += 2.0 * E + 4.0 * S
            # split: read SPL id, edge, two rows (coords, pre-activations, signs), write one row,
            # two edges, two next-crossings, and 2-face keys (32-bit key per slot, hash + entry per key)
            by["split"] += S * (4 + 8 + 3 * (8.0 * D + 8.0 * N + 8.0 * Wd) + 16 + 4) + 4.0 * S * P + 12.0 * Kv
            # sort: linear grouping reads and writes each (key, slot) pair once
            by["sort"] += 16.0 * S * P
            # pair: per key its (key, slot) or table entry, hash and perturbed entry; per pair two face
            # rows, one edge, one next crossing
            by["pair"] += Kv * (8.0 + 12.0) + (Kv / 2) * (2 * 8.0 * (wn + 1) + 8 + 2)
        s0 += N
    return by, flops


def traffic_record(family):
    """HBM bytes per launch measured with rocprofv3 counters, if they were taken
    on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2306_07212_amd", "csrc", "kernels.hip"), "rb").read()
    if rec.get("kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("families", {}).get(family)


def cpu_baseline(net, half=0.06):
    """The CPU oracle (single thread) on the centred sub-box [-half, half]^3 of
    the same network: a bounded sample of the same workload."""
    import oracle
    oracle.build(force=False)
    lo, hi = np.full(3, -half), np.full(3, half)
    t = time.perf_counter()
    r = oracle.extract(net, lo, hi)
    dt = time.perf_counter() - t
    splits = int(r.steps[:, 2].sum())
    return {"value": splits / dt, "unit": "edges subdivided/s", "cores": 1, "kind": "oracle",
            "sample": f"same 3-256-256-256-1 network on the centred sub-box [-{half},{half}]^3 "
                      f"(all 768 neurons): {r.V} vertices, {r.E} edges, {splits} splits in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="plain_large", help="workloads function name (default: the 768-neuron net)")
    ap.add_argument("--pairing", default="hash", choices=["hash", "sort"], help="step-5 grouping of 2-face keys")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU design is documented, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_07212_amd import pcx
    from paper_2306_07212_amd import workloads as wl

    net = getattr(wl, args.workload)()
    D = net.D
    box = wl.cube(D)
    incl = args.workload.startswith("differentiable")
    mlp = pcx.MLP.from_net(net)
    torch.cuda.synchronize()

    def run(timing):
        cx = pcx.extract(mlp, box.lo, box.hi, include_output=incl, timing=timing, pairing=args.pairing)
        return cx

    # warm-up: sizes the buffers (capacity hints) and finds the dominant kernel family
    fam_ms = dict.fromkeys(FAMILIES, 0.0)
    steps = info = None
    for i in range(max(1, args.warmup)):
        t = time.perf_counter()
        cx = run(True)
        info = cx.info()
        steps = cx.steps()
        for f in FAMILIES:
            fam_ms[f] = cx.kernel_time(f)[0]
        cx.close()
        print(f"[bench] warmup {i}: V={info.V} E={info.E} splits={info.total_splits} "
              f"{1e3 * (time.perf_counter() - t):.1f} ms  kernels(ms): "
              + " ".join(f"{f}={fam_ms[f]:.1f}" for f in FAMILIES), file=sys.stderr, flush=True)
    dom = max(FAMILIES, key=lambda f: fam_ms[f])

    # timed region: K extractions, the dominant family timed with HIP events on its stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom_ms, dom_launches = 0.0, 0
    for i in range(args.steps):
        cx = run([dom])
        ms, n = cx.kernel_time(dom)
        dom_ms += ms
        dom_launches += n
        info = cx.info()
        cx.close()
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / args.steps

    by, flops = algorithmic_cost(net.widths, steps, incl)
    avg_launch_s = dom_ms / 1e3 / max(1, dom_launches)
    per_ext_launches = dom_launches / args.steps
    if dom == "gemm":
        achieved = flops / per_ext_launches / avg_launch_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS}
    else:
        achieved = by[dom] / per_ext_launches / avg_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    roof["traffic"] = traffic_record(dom)
    roof["kernel"] = dom
    roof["launches_per_step"] = per_ext_launches
    roof["avg_launch_us"] = avg_launch_s * 1e6

    out = {
        "metric": METRIC,
        "value": info.total_splits / T,
        "unit": "edges subdivided/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain extraction, MLP {'-'.join(map(str, net.widths))} ReLU, "
                               f"He-normal weights, U(-0.5,0.5) biases, box [-1,1]^{D}",
                   "neurons_subdivided": int(info.n_steps), "pairing": args.pairing,
                   "parallelism": "single GPU"},
        "vertices_per_s": info.V / T,
        "edges_per_s": info.E / T,
        "V": info.V, "E": info.E, "splits": info.total_splits, "pairs": info.total_pairs,
        "peak_device_bytes": info.peak_bytes,
        "device_ms_per_step": info.time_ms,
        "kernel_ms_warmup": fam_ms,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(net) if args.workload == "plain_large" else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
