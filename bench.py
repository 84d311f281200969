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
    work of one extraction, from the per-step counters (per-unit figures below)."""
    D = widths[0]
    layers, Wd = layer_table(widths, include_output)
    ZS = max(x["N"] for x in layers)
    P = 2 * (D - 1)
    by = dict.fromkeys(FAMILIES, 0.0)
    flops = 0.0
    s0 = 0
    for li, ly in enumerate(layers):
        N, K, nw = ly["N"], ly["K"], ly["nw"]
        last = li == len(layers) - 1
        V0, E0 = steps[s0, 0], steps[s0, 1]
        kin = D if s0 == 0 else K
        flops += 2.0 * V0 * kin * N
        by["gemm"] += V0 * (8.0 * kin + 8.0 * N + 8.0 * nw)
        by["next"] += E0 * (8.0 + 2 * 8.0 * nw + 2.0)
        for j, st in enumerate(steps[s0:s0 + N]):
            V, E, S, Kv = (float(v) for v in st)
            by["select"] += 2.0 * E + 4.0 * S
            # split: read SPL id, edge, the two endpoint values at neuron j, two rows (coords, carried
            # pre-activations, signs), write one row, two edges, two next-crossings, and 2-face keys
            # (32-bit key per slot, hash + entry per key). Carried columns: all N of the layer (the next
            # layer's evaluation reads them), in the last subdivided layer only the neurons after j.
            Nc = (N - j - 1) if last else N
            by["split"] += S * (4 + 8 + 16 + 3 * (8.0 * D + 8.0 * Nc + 8.0 * Wd) + 16 + 4) + 4.0 * S * P + 12.0 * Kv
            # sort: linear grouping reads and writes each (key, slot) pair once
            by["sort"] += 16.0 * S * P
            # pair: per key slot its 12-byte key read (the scope table's figure); per pair one edge,
            # one next crossing and the sign word at the neuron of both new vertices (the first
            # crossing search); the optional row comparison (2 * 8 (wn + 1) per pair) is not counted
            by["pair"] += Kv * 12.0 + (Kv / 2) * (8.0 + 1.0 + 2 * 8.0)
        s0 += N
    return by, flops


def survey_bytes(widths, steps, include_output=False):
    """Algorithmic bytes of the subdivision steps as the scope table counts them
    (per neuron step n: z column, sign write, edge endpoints, two 2-bit endpoint
    lookups, the split's read of two rows and write of one (coordinates, the
    pre-activations of the neurons after n in its layer, sign words) plus two
    edges, 2-face key write + read, new edges):

        B_n = 8 V_n + V_n/4 + 8 E_n + E_n/2 + S_n [3 (8D + 8 L_n + 8 Wd) + 12] + 24 K_n + 4 K_n

    with L_n = neurons after n in its layer. Returns (sum of B_n, the split's
    share: S_n [3 (8D + 8 L_n + 8 Wd) + 12] + 12 K_n)."""
    D = widths[0]
    layers, Wd = layer_table(widths, include_output)
    total = split = 0.0
    s0 = 0
    for ly in layers:
        N = ly["N"]
        for j, st in enumerate(steps[s0:s0 + N]):
            V, E, S, K = (float(v) for v in st)
            Ln = N - j - 1
            sp = S * (3 * (8.0 * D + 8.0 * Ln + 8.0 * Wd) + 12) + 12.0 * K
            split += sp
            total += 8 * V + V / 4 + 8 * E + E / 2 + sp + 12.0 * K + 4.0 * K
        s0 += N
    return total, split


def host_cpu():
    """CPU model and hardware threads of the host the CPU baseline runs on."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "cpu_count": os.cpu_count()}


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["kernels.hip", "device.h", "internal.h"]
# kernel name prefix -> family (the per-step path's kernels)
KERNEL_FAMILY = {"pcx::k_gemm": "gemm", "pcx::k_next_all": "next", "pcx::k_sel_": "select",
                 "pcx::k_split": "split", "pcx::k_sort_": "sort", "pcx::k_pair": "pair", "pcx::k_hpair_": "pair"}


def kernels_sha256():
    """Digest of the kernel sources' code (comments and blank space dropped, so
    that an edited comment keeps counters taken on the same code valid)."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        src = open(os.path.join(ROOT, "paper_2306_07212_amd", "csrc", f)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def traffic_record(family):
    """HBM bytes per launch of a family's kernels measured with rocprofv3 counters,
    if they were taken on the current kernel source (else None)."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    rec = json.load(open(TRAFFIC_JSON))
    if rec.get("kernels_sha256") != kernels_sha256():
        return None
    fam = rec.get("families", {}).get(family)
    return None if fam is None else fam["bytes_per_launch"]


def pmc_summary(fetch_csv, write_csv):
    """Turns two rocprofv3 --pmc runs of `bench.py --copy-probe` (FETCH_SIZE, then
    WRITE_SIZE) into HBM bytes per launch per kernel family. Each counter is scaled
    by what it reads for the 1 GiB probe copy (2^30 bytes read, 2^30 written)."""
    import csv

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        probe = [float(r["Counter_Value"]) for r in rows
                 if "copyBuffer" in r["Kernel_Name"] and float(r["Counter_Value"]) > 2.0 ** 18]
        if not probe:
            raise SystemExit(f"{path}: no 1 GiB probe copy found (run bench.py with --copy-probe)")
        scale = 2.0 ** 30 / (probe[0] * 1024.0)   # bytes per counter KiB
        # the first extraction of a process grows its storage and redoes the steps
        # that found it too small (launches that do nothing): count the later ones
        inits = [i for i, r in enumerate(rows) if "k_init_box" in r["Kernel_Name"]]
        if len(inits) >= 2:
            rows = rows[inits[1]:]
        per = {}
        for r in rows:
            name = r["Kernel_Name"]
            name = name[5:] if name.startswith("void ") else name  # templates carry their return type
            fam = next((f for k, f in KERNEL_FAMILY.items() if name.startswith(k)), None)
            if fam is None:
                continue
            per.setdefault(fam, []).append(float(r["Counter_Value"]) * 1024.0 * scale)
        return per, scale

    fetch, fs = load(fetch_csv, "FETCH_SIZE")
    write, ws = load(write_csv, "WRITE_SIZE")
    fams = {}
    for f in fetch:
        fams[f] = {"dispatches": len(fetch[f]), "fetch_bytes_per_launch": sum(fetch[f]) / len(fetch[f]),
                   "write_bytes_per_launch": sum(write.get(f, [0.0])) / max(1, len(write.get(f, [])))}
        fams[f]["bytes_per_launch"] = fams[f]["fetch_bytes_per_launch"] + fams[f]["write_bytes_per_launch"]
    return {"kernels_sha256": kernels_sha256(), "fetch_scale_bytes_per_KiB": fs,
            "write_scale_bytes_per_KiB": ws, "families": fams}


def cpu_baseline(net, half=0.08):
    """The CPU oracle on the centred sub-box [-half, half]^3 of the same network
    (a bounded sample of the same workload): on one thread, then with its
    per-vertex loops on all host threads (at most 16)."""
    import oracle
    oracle.build(force=False)
    lo, hi = np.full(3, -half), np.full(3, half)
    t = time.perf_counter()
    r = oracle.extract(net, lo, hi)
    dt = time.perf_counter() - t
    splits = int(r.steps[:, 2].sum())
    hc = host_cpu()
    nth = max(1, min(16, hc["nproc"]))
    t = time.perf_counter()
    oracle.extract(net, lo, hi, threads=nth)
    dtn = time.perf_counter() - t
    return {"value": splits / dt, "unit": "edges subdivided/s", "cores": 1, "kind": "oracle",
            "sample": f"same 3-256-256-256-1 network on the centred sub-box [-{half},{half}]^3 "
                      f"(all 768 neurons): {r.V} vertices, {r.E} edges, {splits} splits in {dt:.1f} s "
                      "on one thread",
            "all_cores": {"value": splits / dtn, "cores": nth, "seconds": dtn,
                          "note": "the oracle's per-vertex loops (evaluation, signs, splits) on all threads; "
                                  "its exact sort of 2-face rows stays sequential"}, **hc}


def pct(v, q):
    return float(np.percentile(np.asarray(v, np.float64), q)) if len(v) else 0.0


def oracle_sample_rate(nets, boxes, threads):
    """Oracle splits/s over a sample of networks on `threads` threads (one network
    per thread at a time: the C oracle runs without the GIL)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=False)
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda nb: oracle.extract(nb[0], nb[1].lo, nb[1].hi), zip(nets, boxes)))
    dt = time.perf_counter() - t
    splits = sum(int(r.steps[:, 2].sum()) for r in res)
    return splits / dt, splits, dt


def form_batched(args, pcx, wl, torch):
    """4096 networks 2-[w]xd-1 in one persistent launch vs the per-step path."""
    nets = wl.batch_nets()
    box = wl.cube(2)
    mlps = [pcx.MLP.from_net(n) for n in nets]
    boxes = [(box.lo, box.hi)] * len(nets)
    tuned = pcx.batch_tune(mlps, boxes)
    for _ in range(max(1, args.warmup)):
        pcx.Batch(mlps, boxes).close()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt = pcx.Batch(mlps, boxes)
        st = bt.stats()
        kms.append(st.kernel_ms)
        bt.close()
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / args.steps
    # algorithmic bytes of every network's steps (the scope table's count), against the launch's time
    bt = pcx.Batch(mlps, boxes)
    b8 = sum(survey_bytes(n.widths, bt.steps(i))[0] for i, n in enumerate(nets))
    bt.close()
    k_med = float(np.median(kms)) / 1e3
    achieved = b8 / k_med / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": b8, "kernel": "pcx::k_batch",
            "launches_per_step": 1, "avg_launch_us": k_med * 1e6, "traffic": None,
            "bytes_rule": "scope-table count summed over every network's steps; the launch also evaluates "
                          "every layer (FP64 MFMA for layers of up to 64 neurons, not in the count)"}
    # per-step path (ordinary per-step kernels, each network once) on a stratified sample
    os.environ["PCX_NO_TINY"] = "1"
    os.environ["PCX_NO_GRAPH"] = "1"
    sample = list(range(0, len(nets), 16))
    t1 = time.perf_counter()
    s_splits = 0
    for i in sample:
        cx = pcx.extract(mlps[i], box.lo, box.hi)
        s_splits += cx.info().total_splits
        cx.close()
    t_sample = time.perf_counter() - t1
    del os.environ["PCX_NO_TINY"], os.environ["PCX_NO_GRAPH"]
    plain_rate = s_splits / t_sample
    out = {"metric": METRIC, "value": st.total_splits / T, "unit": "edges subdivided/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": T * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batched: 4096 MLPs 2-[w]xd-1, w in {8,16,32,64}, d in {2,3,4}, seeds (3, i), "
                                  "box [-1,1]^2, one persistent launch", "parallelism": "single GPU"},
           "vertices_per_s": st.total_V / T, "edges_per_s": st.total_E / T, "V": st.total_V, "E": st.total_E,
           "splits": st.total_splits, "kernel_ms": float(np.median(kms)), "workgroups": st.workgroups,
           "tuned": tuned, "fallbacks": st.fallbacks, "roofline": roof,
           "plain_path": {"edges_subdivided_per_s": plain_rate, "sample": f"{len(sample)} of 4096 networks "
                          f"extracted one by one on the per-step kernels in {t_sample:.2f} s"},
           "speedup_vs_plain": (st.total_splits / T) / plain_rate}
    if not args.no_cpu_baseline:
        osample = list(range(0, len(nets), 8))
        snets = [nets[i] for i in osample]
        sboxes = [box] * len(snets)
        r1, sp1, dt1 = oracle_sample_rate(snets, sboxes, 1)
        hc = host_cpu()
        nth = min(16, hc["nproc"])
        rn, spn, dtn = oracle_sample_rate(snets, sboxes, nth)
        out["cpu_baseline"] = {"value": rn, "unit": "edges subdivided/s", "cores": nth, "kind": "oracle",
                               "sample": f"{len(osample)} of 4096 networks (every 8th), one network per thread: "
                                         f"{spn} splits in {dtn:.2f} s", "single_core": {"value": r1, "cores": 1,
                                         "seconds": dt1}, **hc}
    return out


def form_configs(args, pcx, wl, torch):
    """The small configurations against the CPU oracle (one core): the
    2-8-8-1 and the 3-64-64-64-1 (with its output) networks whole, the 4096
    batched networks on a stratified sample; the GPU side as the library runs
    each (per-step path, batched kernel). The 768-neuron network is the plain
    bench line."""
    import oracle
    oracle.build(force=False)

    def gpu_single(net, incl):
        m = pcx.MLP.from_net(net)
        box = wl.cube(net.D)
        for _ in range(max(1, args.warmup)):
            pcx.extract(m, box.lo, box.hi, include_output=incl).close()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(1, args.steps)):
            t = time.perf_counter()
            cx = pcx.extract(m, box.lo, box.hi, include_output=incl)
            info = cx.info()
            cx.close()
            ts.append(time.perf_counter() - t)
        m.close()
        return float(np.median(ts)), info

    rows = {}
    for key, name, incl in (("C1", "plain_small", False), ("C5", "differentiable", True)):
        net = getattr(wl, name)()
        box = wl.cube(net.D)
        T, info = gpu_single(net, incl)
        t = time.perf_counter()
        r = oracle.extract(net, box.lo, box.hi, include_output=incl)
        To = time.perf_counter() - t
        splits = int(r.steps[:, 2].sum())
        assert (r.V, r.E) == (info.V, info.E)
        rows[key] = {"network": "-".join(map(str, net.widths)), "V": info.V, "E": info.E, "splits": splits,
                     "gpu_ms": T * 1e3, "oracle_1core_ms": To * 1e3, "speedup": To / T,
                     "gpu_edges_subdivided_per_s": splits / T}
    # C3: the batched kernel on all 4096 networks; the oracle on every 64th one
    nets = wl.batch_nets()
    box = wl.cube(2)
    mlps = [pcx.MLP.from_net(n) for n in nets]
    boxes = [(box.lo, box.hi)] * len(nets)
    for _ in range(max(1, args.warmup)):
        pcx.Batch(mlps, boxes).close()
    torch.cuda.synchronize()
    ts = []
    for _ in range(max(1, args.steps)):
        t = time.perf_counter()
        bt = pcx.Batch(mlps, boxes)
        st = bt.stats()
        bt.close()
        ts.append(time.perf_counter() - t)
    for m in mlps:
        m.close()
    T = float(np.median(ts))
    sample = range(0, len(nets), 64)
    t = time.perf_counter()
    o_splits = 0
    for i in sample:
        o_splits += int(oracle.extract(nets[i], box.lo, box.hi).steps[:, 2].sum())
    To = time.perf_counter() - t
    gpu_rate, o_rate = st.total_splits / T, o_splits / To
    rows["C3"] = {"network": "4096 x 2-[w]xd-1", "V": st.total_V, "E": st.total_E, "splits": st.total_splits,
                  "gpu_ms": T * 1e3, "gpu_edges_subdivided_per_s": gpu_rate,
                  "oracle_1core_edges_subdivided_per_s": o_rate, "oracle_sample": f"{len(sample)} of 4096 networks "
                  f"({o_splits} splits in {To:.2f} s)", "speedup": gpu_rate / o_rate}
    return {"metric": METRIC, "value": rows["C5"]["gpu_edges_subdivided_per_s"], "unit": "edges subdivided/s (C5)",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": rows["C5"]["gpu_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "small configurations against the CPU oracle (one core): 2-8-8-1, "
                                   "3-64-64-64-1 with its output, 4096 batched networks", "parallelism": "single GPU"},
            "configs": rows}


def form_served(args, pcx, wl, torch):
    """Poisson stream of 2000 requests (D in {2,3}, widths 16-128, depths 2-4):
    continuous batching vs the per-step path as a FIFO single server."""
    reqs = wl.serve_requests(2000, rate_per_s=1.0)
    unit = np.array([r.arrival_s for r in reqs])          # unit-rate arrival times
    mlps = [pcx.MLP.from_net(r.net) for r in reqs]
    # the per-step path as the server's own workers run it (no graph replay of repeated requests)
    os.environ["PCX_NO_GRAPH"] = "1"
    for r, m in zip(reqs[:100], mlps[:100]):  # warm the device memory pool
        pcx.extract(m, r.box.lo, r.box.hi).close()
    # per-step path: service time of every request alone
    svc = np.empty(len(reqs))
    alone = np.empty((len(reqs), 3), np.int64)  # V, E, splits of each request extracted alone
    for i, (r, m) in enumerate(zip(reqs, mlps)):
        t = time.perf_counter()
        cx = pcx.extract(m, r.box.lo, r.box.hi)
        info = cx.info()
        cx.close()
        svc[i] = time.perf_counter() - t
        alone[i] = (info.V, info.E, info.total_splits)
        if i % 250 == 0:
            print(f"[bench] served: plain service times {i}/{len(reqs)}", file=sys.stderr, flush=True)
    mu = len(reqs) / svc.sum()  # saturation throughput of the per-step path (requests/s)
    out_rates = []
    for f in (0.25, 0.5, 1.0, 1.5, 2.0):
        lam = f * mu
        arr = unit / lam
        # FIFO single server with the measured service times (the per-step path, one request at a time)
        fin = np.empty(len(reqs))
        tcur = 0.0
        for i in range(len(reqs)):
            tcur = max(tcur, arr[i]) + svc[i]
            fin[i] = tcur
        lat_plain = (fin - arr) * 1e3
        srv = pcx.Server()
        t0 = time.perf_counter()
        tickets = []
        res = [None] * len(reqs)
        failed = []

        # a client consumes each result as it completes (in submission order) and releases it, as a
        # serving loop would: finished complexes are the caller's memory until released
        def consume():
            for i in range(len(reqs)):
                while i >= len(tickets):
                    time.sleep(1e-4)
                tk = tickets[i]
                res[i] = srv.wait(tk)
                if res[i]["status"] != 0:
                    failed.append((i, res[i]["status"], srv.error(tk)))
                srv.release(tk)

        import threading
        th = threading.Thread(target=consume)
        th.start()
        for a, r, m in zip(arr, reqs, mlps):
            dt = a - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(m, r.box.lo, r.box.hi))
        th.join()
        st = srv.stats()
        srv.close()
        if failed:
            print(f"[bench] served: {len(failed)} requests failed, first: {failed[:3]}", file=sys.stderr, flush=True)
            raise SystemExit(f"served requests failed: {failed[:3]}")
        got = np.array([(x["V"], x["E"], x["total_splits"]) for x in res], np.int64)
        bad = np.nonzero(np.any(got != alone, axis=1))[0]
        if len(bad):
            raise SystemExit(f"served results differ from the same requests extracted alone: {bad[:5].tolist()}")
        live = None
        if f in (1.0, 2.0):
            # the per-step path as a live FIFO single server under the same arrivals
            lat = np.empty(len(reqs))
            t0 = time.perf_counter()
            for i, (a, r, m) in enumerate(zip(arr, reqs, mlps)):
                dt = a - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                cx = pcx.extract(m, r.box.lo, r.box.hi)
                cx.close()
                lat[i] = (time.perf_counter() - t0 - a) * 1e3
                if i % 500 == 0:
                    print(f"[bench] served: live FIFO {i}/{len(reqs)}", file=sys.stderr, flush=True)
            live = {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "jobs_per_s": len(reqs) / (time.perf_counter() - t0)}
        out_rates.append({"rate_x_plain_saturation": f, "rate_per_s": lam,
                          "served": {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "jobs_per_s": st["jobs_per_s"],
                                     "splits_per_s": st["splits_per_s"], "ticks": st["ticks"],
                                     "mean_tick_jobs": st["mean_tick_jobs"],
                                     "batched_fraction": float(np.mean([x["batched"] for x in res]))},
                          "plain_fifo": {"p50_ms": pct(lat_plain, 50), "p99_ms": pct(lat_plain, 99),
                                         "jobs_per_s": len(reqs) / fin[-1],
                                         "from": "queue of the measured alone service times"},
                          "plain_fifo_live": live, "results_checked": len(reqs)})
        print(f"[bench] served rate {f}x: {json.dumps(out_rates[-1])}", file=sys.stderr, flush=True)
    mid = out_rates[2]
    out = {"metric": METRIC, "value": mid["served"]["p99_ms"], "unit": "ms (p99 latency at the plain path's "
           "saturation rate)", "n_gpus": 1, "steps": len(reqs), "warmup": 0, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "served: Poisson stream of 2000 requests, D in {2,3}, constant width U[16,128], "
                                  "depth U{2,3,4}, box [-1,1]^D, seeds (4, i)", "parallelism": "single GPU"},
           "plain_saturation_req_per_s": mu, "plain_mean_service_ms": float(svc.mean() * 1e3),
           "plain_service_ms": {"p50": pct(svc * 1e3, 50), "p99": pct(svc * 1e3, 99)}, "rates": out_rates}
    del os.environ["PCX_NO_GRAPH"]
    if not args.no_cpu_baseline:
        # the oracle's service times (one core) on every 10th request among those with at most
        # 20K splits (the largest requests would take the oracle minutes each), beside the GPU
        # per-step path's alone service times on the same requests; then the oracle's throughput
        # on that subset with one request per thread on all host cores
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        oracle.build(force=False)
        sample = [i for i in range(0, len(reqs), 10) if alone[i, 2] <= 20000]
        ts = []
        for k, i in enumerate(sample):
            t = time.perf_counter()
            oracle.extract(reqs[i].net, reqs[i].box.lo, reqs[i].box.hi)
            ts.append(time.perf_counter() - t)
            if k % 40 == 0:
                print(f"[bench] served: oracle {k}/{len(sample)}", file=sys.stderr, flush=True)
        ts = np.array(ts) * 1e3
        hc = host_cpu()
        nth = min(16, hc["nproc"])
        t = time.perf_counter()
        with ThreadPoolExecutor(max_workers=nth) as ex:
            list(ex.map(lambda i: oracle.extract(reqs[i].net, reqs[i].box.lo, reqs[i].box.hi), sample))
        dt = time.perf_counter() - t
        g = svc[sample] * 1e3
        out["cpu_baseline"] = {"value": float(np.percentile(ts, 99)), "unit": "ms (p99 service time, one core, "
                               "no queueing)", "cores": 1, "kind": "oracle",
                               "sample": f"{len(sample)} requests: every 10th of the 2000 with at most 20000 "
                                         f"splits (of {len(range(0, len(reqs), 10))})",
                               "p50_ms": float(np.percentile(ts, 50)), "mean_ms": float(ts.mean()),
                               "gpu_plain_same_requests": {"p50_ms": pct(g, 50), "p99_ms": pct(g, 99),
                                                           "mean_ms": float(g.mean())},
                               "all_cores": {"cores": nth, "requests_per_s": len(sample) / dt}, **hc}
    return out


def form_backward(args, pcx, wl, torch):
    """3-64-64-64-1 level set: extraction with tape + loss + hand-written backward."""
    from paper_2306_07212_amd import torch_ops as T
    net = wl.differentiable()
    box = wl.cube(3)
    dev = torch.device("cuda:0")
    res = {}
    grads = {}
    for prec in ("f64", "f32"):
        Ws = [torch.tensor(w, dtype=torch.float64, device=dev, requires_grad=True) for w in net.W]
        bs = [torch.tensor(x, dtype=torch.float64, device=dev, requires_grad=True) for x in net.b]
        for it in range(args.warmup + args.steps):
            if it == args.warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                tb = 0.0
            for p in Ws + bs:
                p.grad = None
            X, SG, Ed = T.extract_coords(Ws, bs, box.lo, box.hi, include_output=True, precision=prec)
            loss = T.level_set_edge_loss(X, SG, Ed, net.widths)
            torch.cuda.synchronize()
            tb0 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            if it >= args.warmup:
                tb += time.perf_counter() - tb0
        T_all = (time.perf_counter() - t0) / args.steps
        grads[prec] = [p.grad.detach().cpu().numpy() for p in Ws + bs]
        res[prec] = {"ms_per_step": T_all * 1e3, "backward_ms": tb / args.steps * 1e3, "V": int(X.shape[0])}
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(grads["f32"], grads["f64"]))
    den = sum(float(np.sum(b ** 2)) for b in grads["f64"])
    V = res["f64"]["V"]
    return {"metric": METRIC, "value": V / (res["f32"]["ms_per_step"] / 1e3), "unit": "vertices/s (extract + loss "
            "+ FP32 backward)", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": res["f32"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64 forward, f32 backward", "data": "synthetic",
            "config": {"workload": "differentiable: MLP 3-64-64-64-1 with the output's level set, loss = sum of "
                                   "squared lengths of level-set edges, box [-1,1]^3", "parallelism": "single GPU"},
            "fp64": res["f64"], "fp32": res["f32"], "fp32_rel_error_vs_fp64": (num / den) ** 0.5}


def form_levelset(args, pcx, wl, torch):
    """Level-set extraction (the output neuron subdivided last) with pruning during
    subdivision (Sec. 5.4.2) against the full extraction, on the 3-64-64-64-1 and
    the 3-256-256-256-1 networks. Both on the per-step kernels: a pruned
    extraction is never replayed from a graph, so the full one is not either."""
    os.environ["PCX_NO_GRAPH"] = "1"
    out = {}
    for name in ("differentiable", "plain_large"):
        net = getattr(wl, name)()
        box = wl.cube(net.D)
        m = pcx.MLP.from_net(net)
        res = {}
        for prune in (False, True):
            for _ in range(max(1, args.warmup)):
                pcx.extract(m, box.lo, box.hi, include_output=True, prune=prune).close()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                cx = pcx.extract(m, box.lo, box.hi, include_output=True, prune=prune)
                inf = cx.info()
                steps = cx.steps()
                cx.close()
            torch.cuda.synchronize()
            T = (time.perf_counter() - t0) / args.steps
            starts, s0 = [], 0
            for n in net.widths[1:]:
                starts.append([int(steps[s0, 0]), int(steps[s0, 1])])
                s0 += n
            res["pruned" if prune else "full"] = {"ms": T * 1e3, "V": inf.V, "E": inf.E,
                                                  "splits": inf.total_splits, "layer_starts_V_E": starts}
            print(f"[bench] levelset {name} prune={prune}: {T * 1e3:.1f} ms V={inf.V} E={inf.E}", file=sys.stderr,
                  flush=True)
        m.close()
        res["speedup"] = res["full"]["ms"] / res["pruned"]["ms"]
        out[name] = res
    del os.environ["PCX_NO_GRAPH"]
    big = out["plain_large"]
    return {"metric": METRIC, "value": big["pruned"]["splits"] / (big["pruned"]["ms"] / 1e3),
            "unit": "edges subdivided/s (pruned level-set extraction)", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": big["pruned"]["ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "level set of the output of MLP 3-256-256-256-1 (and 3-64-64-64-1), box [-1,1]^3, "
                                   "pruning during subdivision vs full extraction", "parallelism": "single GPU"},
            "results": out}


def form_simplex(args, pcx, wl, torch):
    """Hypercube vs simplex domain of the same volume (Sec. 5.2: the simplex has
    D + 1 corners instead of 2^D): an MLP 6-32-32-1, seeds 6."""
    import math
    D = 6
    net = wl.he_mlp([D, 32, 32, 1], 6)
    m = pcx.MLP.from_net(net)
    box = wl.cube(D)
    s = 2.0 * math.factorial(D) ** (1.0 / D)
    corners = np.vstack([-np.ones(D)] + [-np.ones(D) + s * np.eye(D)[i] for i in range(D)])
    res = {}
    for name, run in (("hypercube", lambda: pcx.extract(m, box.lo, box.hi)),
                      ("simplex", lambda: pcx.extract_simplex(m, corners))):
        for _ in range(max(1, args.warmup)):
            run().close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            cx = run()
            inf = cx.info()
            cx.close()
        torch.cuda.synchronize()
        T = (time.perf_counter() - t0) / args.steps
        cx = run()
        S = cx.signs()
        cx.close()
        mdom = 2 * D if name == "hypercube" else D + 1
        boundary = int(np.any(S[:, :mdom] == 0, axis=1).sum())
        res[name] = {"ms": T * 1e3, "V": inf.V, "E": inf.E, "splits": inf.total_splits,
                     "boundary_vertices": boundary, "interior_vertices": inf.V - boundary}
        print(f"[bench] simplex form {name}: {json.dumps(res[name])}", file=sys.stderr, flush=True)
    m.close()
    sp = res["simplex"]
    return {"metric": METRIC, "value": sp["splits"] / (sp["ms"] / 1e3), "unit": "edges subdivided/s (simplex domain)",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sp["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "MLP 6-32-32-1 (seed 6) on [-1,1]^6 vs the corner simplex of equal volume",
                       "parallelism": "single GPU"}, "results": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="plain_large", help="workloads function name (default: the 768-neuron net)")
    ap.add_argument("--pairing", default="hash", choices=["hash", "sort"], help="step-5 grouping of 2-face keys")
    ap.add_argument("--form", default="plain",
                    choices=["plain", "batched", "served", "backward", "levelset", "simplex", "configs"],
                    help="plain (default): one large network; the others measure the systems forms")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one 1 GiB device copy (reads 1 GiB, writes 1 GiB): the reference for "
                         "scaling hardware traffic counters")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: turn the counter CSVs of two rocprofv3 --pmc runs of this script (with "
                         "--copy-probe) into profiles/traffic.json")
    args = ap.parse_args()
    if args.pmc_summary:
        rec = pmc_summary(*args.pmc_summary)
        rec["sources"] = args.pmc_summary
        json.dump(rec, open(TRAFFIC_JSON, "w"), indent=1)
        print(json.dumps(rec, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU design is documented, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_07212_amd import pcx
    from paper_2306_07212_amd import workloads as wl

    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.form != "plain":
        fn = {"batched": form_batched, "served": form_served, "backward": form_backward,
              "levelset": form_levelset, "simplex": form_simplex, "configs": form_configs}[args.form]
        print(json.dumps(fn(args, pcx, wl, torch)), flush=True)
        return

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
              + " ".join(f"{f}={fam_ms[f]:.1f}" for f in FAMILIES)
              + ("  (every launch timed; this first run also creates the HIP events later runs reuse)"
                 if i == 0 else ""), file=sys.stderr, flush=True)
    dom = max(FAMILIES, key=lambda f: fam_ms[f])

    # timed region: K extractions; in the last one every launch of the dominant
    # family records HIP events on its stream (each timed launch costs a few
    # microseconds of stream time, so the other K-1 run without them)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom_ms, dom_launches = 0.0, 0
    for i in range(args.steps):
        timed = i == args.steps - 1
        cx = run([dom] if timed else False)
        if timed:
            dom_ms, dom_launches = cx.kernel_time(dom)
        info = cx.info()
        cx.close()
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / args.steps
    # outside the timed region: one extraction followed by the copy of the complex to host memory
    t1 = time.perf_counter()
    cx = run(False)
    cx.copy()
    cx.close()
    T_d2h = time.perf_counter() - t1
    # outside the timed region: every family timed in each of R extractions (per-family medians)
    R = 10
    runs = []
    for _ in range(R):
        cx = run(True)
        runs.append({f: cx.kernel_time(f) for f in FAMILIES})
        cx.close()
    med_ms = {f: float(np.median([r[f][0] for r in runs])) for f in FAMILIES}
    med_launch_s = {f: float(np.median([r[f][0] / 1e3 / max(1, r[f][1]) for r in runs])) for f in FAMILIES}

    by, flops = algorithmic_cost(net.widths, steps, incl)
    b8_total, b8_split = survey_bytes(net.widths, steps, incl)
    avg_launch_s = dom_ms / 1e3 / max(1, dom_launches)
    per_ext_launches = dom_launches
    if dom == "gemm":
        achieved = flops / per_ext_launches / avg_launch_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS,
                "flop_per_launch": flops / per_ext_launches}
    else:
        # the scope table's count: for the split, L_n = neurons after n in its layer
        per_launch = (b8_split if dom == "split" else by[dom]) / per_ext_launches
        achieved = per_launch / avg_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": per_launch,
                "bytes_rule": "scope-table count: S_n [3 (8D + 8 L_n + 8 Wd) + 12] + 12 K_n per step"
                if dom == "split" else "per-unit figures of the kernel family"}
        roof["frac_median_of_runs"] = per_launch / med_launch_s[dom] / 1e9 / HBM_PEAK_GBS
        if dom == "split":
            # the same launches counted with every carried pre-activation column the split moves
            # (all N of the layer except in the last subdivided layer: the next evaluation reads them)
            cpl = by["split"] / per_ext_launches
            roof["carried_columns"] = {"bytes_per_launch": cpl, "achieved": cpl / avg_launch_s / 1e9,
                                       "frac": cpl / avg_launch_s / 1e9 / HBM_PEAK_GBS}
            # the per-layer sums the count needs: bytes = sum over layers of
            # (3 (8D + 8 Wd) + 12) sum_S + 24 sum_S_Ln + 12 sum_K
            layers, Wd_ = layer_table(net.widths, incl)
            terms, s0 = [], 0
            for ly in layers:
                blk = np.asarray(steps[s0:s0 + ly["N"]], np.float64)
                Ln = ly["N"] - 1 - np.arange(len(blk))
                terms.append({"N": ly["N"], "sum_S": int(blk[:, 2].sum()), "sum_S_Ln": int((blk[:, 2] * Ln).sum()),
                              "sum_K": int(blk[:, 3].sum())})
                s0 += ly["N"]
            roof["scope_terms"] = {"D": D, "Wd": Wd_, "layers": terms}
    # every family, from the per-family medians of the R extractions with all families timed
    fam_roof = {}
    for f in FAMILIES:
        if med_ms[f] <= 0:
            continue
        s_ = med_ms[f] / 1e3
        fam_roof[f] = {"ms": med_ms[f], "GB_per_s": by[f] / s_ / 1e9, "hbm_frac": by[f] / s_ / 1e9 / HBM_PEAK_GBS,
                       "avg_launch_us": med_launch_s[f] * 1e6}
        if f == "gemm":
            fam_roof[f]["TFLOP_per_s"] = flops / s_ / 1e12
            fam_roof[f]["mfma_frac"] = flops / s_ / 1e12 / FP64_PEAK_TFLOPS
        if f == "pair":
            fam_roof[f]["note"] = ("12 B per key slot and 25 B per pair (edge, next crossing, one sign word of each "
                                   "new vertex); two launches per neuron of a few microseconds each, so latency, "
                                   "not bytes, bounds it")
    sub_ms = sum(med_ms[f] for f in ("next", "select", "split", "sort", "pair"))
    subdivision = {"bytes": b8_total, "ms": sub_ms, "GB_per_s": b8_total / (sub_ms / 1e3) / 1e9,
                   "hbm_frac": b8_total / (sub_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                   "kernels": "first-crossing scan, compaction, split, pairing (steps 2-5), medians of "
                              f"{R} extractions"}
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
        "edge_sign_tests_per_s": float(steps[:, 1].sum()) / T,
        "ms_with_copy_to_host": T_d2h * 1e3,
        "V": info.V, "E": info.E, "splits": info.total_splits, "pairs": info.total_pairs,
        "peak_device_bytes": info.peak_bytes,
        "device_ms_per_step": info.time_ms,
        "kernel_ms_warmup": fam_ms,
        "roofline": roof,
        "subdivision": subdivision,
        "families": fam_roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(net) if args.workload == "plain_large" else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
