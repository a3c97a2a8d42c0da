#!/usr/bin/env python3
"""Benchmark of the MI355X butterfly-peeling path.

A step is one tip decomposition of both sides (U, then V) of the seeded
Chung-Lu workload |U|=1M, |V|=200k, 20M edges, exponent 2.1, degree cap 50k,
P=150, plain bound rule: preprocessing, priority counting, coarse-grained
peel rounds (with recounts) and the fine-grained persistent kernel, all on the
GPU with the graph resident in HBM before the timed region.

Prints one JSON line: wedges/s over the whole step (value), the per-step
decomposition time, the roofline of the dominant kernel class (algorithmic
bytes / its HIP-event time on the library's stream), and the CPU oracle timed
on a bounded sample of the same workload family.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME]
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

METRIC = "wedges/s + tip/wing decomposition time, learned vs plain CD bounds, 1 GPU"
HBM_PEAK_GBS = 8000.0
# kernel behind each timed class that holds a single kernel
CLASS_KERNEL = {"tip_hrange": "k_tip_peel_hrange<14>", "tip_tiled": "k_tip_peel_tiled<16>", "fd": "k_tip_fd / k_wing_fd",
                "dense": "m_gram"}

WORKLOADS = {
    # name: (graph config, kind, P); kinds: tip (both sides), tip_u (side U),
    # wing (all edges), batch (tip of side U and wing of every graph of a list,
    # one batched call each)
    "tip_cl_1m_200k_20m": ("cl_1m_200k_20m", "tip", 150),
    "tip_cl_500k_100k_5m": ("cl_500k_100k_5m", "tip", 150),
    "wing_cl_500k_100k_5m": ("cl_500k_100k_5m", "wing", 400),
    "tip_er_2k_1k_20k": ("er_2k_1k_20k", "tip", 8),
    "tip_u_cl_5m_1m_100m": ("cl_5m_1m_100m", "tip_u", 150),
    "batch_mixed_1024": ("mixed_1024", "batch", 0),
}
# batch lists: (number of graphs, smallest and largest edge count)
BATCHES = {"mixed_1024": (1024, 1e3, 1e5)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def golden(workload, quantity):
    p = os.path.join(ROOT, "tests", "golden", f"{workload}__{quantity}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)


def run_step(pb, ctx, dg, kind, P, flags):
    """One pass of the hot path; returns (outputs, list of stats dicts)."""
    opts = pb.make_opts(P=P, flags=flags)
    outs, stats = [], []
    if kind in ("tip", "tip_u"):
        for side in ((pb.SIDE_U, pb.SIDE_V) if kind == "tip" else (pb.SIDE_U,)):
            outs.append(pb.tip(ctx, dg, side, opts))
            stats.append(ctx.stats())
    elif kind == "batch":
        outs.append(pb.tip_batch(ctx, dg, pb.SIDE_U, opts))
        stats.append(ctx.stats())
        outs.append(pb.wing_batch(ctx, dg, opts))
        stats.append(ctx.stats())
    else:
        outs.append(pb.wing(ctx, dg, opts))
        stats.append(ctx.stats())
    return outs, stats


def copy_probe(torch, mib=1024, reps=5):
    """Bandwidth of a plain elementwise copy kernel (int32 negate: mib MiB read,
    mib MiB written per launch), timed with events on torch's stream.  Its
    hardware byte counters calibrate those of the path's kernels."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return dict(kernel="int32 negate", bytes_per_launch=2 * mib * (1 << 20), ms=round(ms, 4),
                gbs=round(2 * mib * (1 << 20) / (ms / 1e3) / 1e9, 1))


def profile_traffic(kernel_class, workload):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel's), or
    None when there is none or the kernel's sources changed since."""
    import re

    names = {"tip_hrange": "k_tip_peel_hrange", "tip_tiled": "k_tip_peel_tiled"}
    if kernel_class not in names:
        return None
    path = os.path.join(ROOT, "profiles", f"{names[kernel_class]}__{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    h = re.search(r"source_sha256: ([0-9a-f]+)", text)
    if not m or not h:
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2110_12511_amd", "csrc", f), "rb").read()
                   for f in ("tip.hip", "dev_common.h"))
    if hashlib.sha256(src).hexdigest() != h.group(1):
        return None
    return int(m.group(1))


def cpu_baseline(graph_cfg, kind, budget_s):
    """The oracle on a bounded sample: the same generator family scaled down
    until one run takes about budget_s seconds on one host core."""
    import oracle
    import synth

    if kind == "batch":
        # the batch's own graphs in order until the budget is spent
        nb, m_min, m_max = BATCHES[graph_cfg]
        wedges, dt, k = 0, 0.0, 0
        while k < nb and dt * 2 < budget_s:
            g = synth.mixed_graph(k, m_min, m_max)
            t0 = time.perf_counter()
            _, st = oracle.tip(g, 0, return_stats=True)
            dt += time.perf_counter() - t0
            wedges += 2 * st["wedges"]
            k += 1
        return dict(value=wedges / dt if dt > 0 else 0.0, unit="wedges/s", cores=1, kind="oracle",
                    sample=f"the first {k} graphs of the batch: tip side U by sequential bottom-up peeling, "
                           f"{wedges} wedges in {dt:.2f} s", seconds=round(dt, 2))
    c = dict(synth.CONFIGS[graph_cfg])
    gen = c.pop("kind")
    scale = 64
    best = None
    while scale >= 1:
        kw = dict(c)
        for k in ("n_u", "n_v", "m"):
            kw[k] = max(1, int(c[k] // scale))
        if gen == "cl":
            kw["cap"] = max(8, c["cap"] // scale)
        g = synth.er(**kw) if gen == "er" else synth.chung_lu(**kw)
        t0 = time.perf_counter()
        if kind in ("tip", "tip_u"):
            _, st = oracle.tip(g, 0, return_stats=True)
            # counting walks the same wedges as peeling without graph updates
            wedges = 2 * st["wedges"]
        else:
            _, st = oracle.wing(g, return_stats=True)
            wedges = st["wedges"]
        dt = time.perf_counter() - t0
        best = dict(value=wedges / dt if dt > 0 else 0.0, unit="wedges/s", cores=1, kind="oracle",
                    sample=f"{g.name}: {kind} side U by sequential bottom-up peeling, {wedges} wedges in {dt:.2f} s "
                           f"(workload scaled 1/{scale})", seconds=round(dt, 2))
        if dt * 4 > budget_s or scale == 1:
            break
        scale //= 2
    return best


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tip_cl_1m_200k_20m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain bound comparison")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    import paper_2110_12511_amd as pb
    import synth

    graph_cfg, kind, P = WORKLOADS[args.workload]
    log(f"[bench] generating {graph_cfg}")
    if kind == "batch":
        nb, m_min, m_max = BATCHES[graph_cfg]
        graphs = [synth.mixed_graph(i, m_min, m_max) for i in range(nb)]
        g = synth.Graph(n_u=sum(x.n_u for x in graphs), n_v=sum(x.n_v for x in graphs),
                        row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
                        name=f"{nb} graphs, m log-uniform in [{m_min:.0e}, {m_max:.0e}], half ER half CL")
        g_m = sum(x.m for x in graphs)
    else:
        g = synth.config_graph(graph_cfg, log=log)
        g_m = g.m
    log(f"[bench] graph {g.name}: m={g_m}")
    ctx = pb.Context()
    if kind == "batch":
        dg = [pb.DeviceGraph.from_graph(x) for x in graphs]
    else:
        dg = pb.DeviceGraph.from_graph(g)
    torch.cuda.synchronize()
    copy = copy_probe(torch)
    log(f"[bench] copy kernel: {copy['gbs']} GB/s")

    for i in range(args.warmup):
        run_step(pb, ctx, dg, kind, P, 0)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")

    step_ms, all_stats, outs = [], [], None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        outs, stats = run_step(pb, ctx, dg, kind, P, pb.binding.F_KERNEL_TIMING)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        all_stats.append(stats)
        log(f"[bench] step {i + 1}/{args.steps}: {step_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_all

    wedges_per_step = [sum(s["wedges"] for s in st) for st in all_stats]
    value = sum(wedges_per_step) / total_s
    ms_per_step = total_s * 1e3 / args.steps

    # dominant kernel class over the timed steps
    agg = {}
    for st in all_stats:
        for s in st:
            for name, k in s["kstat"].items():
                a = agg.setdefault(name, dict(ms=0.0, launches=0, bytes=0, wedges=0))
                for f in a:
                    a[f] += k[f]
    dom = max(agg, key=lambda n: agg[n]["ms"])
    d = agg[dom]
    achieved = d["bytes"] / (d["ms"] / 1e3) / 1e9 if d["ms"] > 0 else 0.0
    roofline = dict(bound="hbm", kernel=CLASS_KERNEL.get(dom, dom), kernel_class=dom, achieved=round(achieved, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=profile_traffic(dom, args.workload),
                    avg_launch_ms=round(d["ms"] / max(d["launches"], 1), 4), launches=d["launches"],
                    algorithmic_bytes=d["bytes"], wedges=d["wedges"],
                    kernel_wedges_per_s=round(d["wedges"] / (d["ms"] / 1e3), 1) if d["ms"] > 0 else 0.0)

    # parity evidence against stored oracle results (when present)
    parity = {}
    qnames = {"tip": ["tip_u", "tip_v"], "tip_u": ["tip_u"], "wing": ["wing"]}.get(kind, [])
    for q, t in zip(qnames, outs):
        rec = golden(graph_cfg, q)
        if rec is not None:
            parity[q] = digest(pb.to_numpy_u64(t)) == rec["sha256"]

    last = all_stats[-1]
    phases = [{k: round(s[k], 2) for k in ("ms_total", "ms_prep", "ms_count", "ms_cd", "ms_fd_prep", "ms_fd")}
              for s in last]
    work = [{k: s[k] for k in ("wedges", "wedges_count", "wedges_cd", "wedges_fd", "rho", "recounts", "partitions",
                                "P_used", "fd_work_max", "fd_work_sum", "updates", "links", "blooms")} for s in last]

    # learned vs plain range bounds on the same graph and P, outside the timed
    # steps (tip workloads, when a trained predictor is stored)
    learned = None
    if kind in ("tip", "tip_u") and not args.no_learned:
        from paper_2110_12511_amd import predictor

        if predictor.install(ctx):
            learned = {}
            for rule_name, rule in (("plain", pb.BOUND_PLAIN), ("learned", pb.BOUND_LEARNED)):
                per_side = []
                for side in ((pb.SIDE_U, pb.SIDE_V) if kind == "tip" else (pb.SIDE_U,)):
                    t = pb.tip(ctx, dg, side, pb.make_opts(P=P, bound_rule=rule))
                    torch.cuda.synchronize()
                    st = ctx.stats()
                    q = "tip_u" if side == pb.SIDE_U else "tip_v"
                    rec = golden(graph_cfg, q)
                    imb = st["fd_work_max"] / max(st["fd_work_sum"] / max(st["partitions"], 1), 1)
                    per_side.append(dict(side=q, ms_total=round(st["ms_total"], 2), ms_cd=round(st["ms_cd"], 2),
                                         ms_fd=round(st["ms_fd"], 2), rho=st["rho"], partitions=st["partitions"],
                                         fd_imbalance=round(imb, 2), rule_used=st["bound_rule_used"],
                                         exact=(digest(pb.to_numpy_u64(t)) == rec["sha256"]) if rec else None))
                learned[rule_name] = per_side

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(graph_cfg, kind, args.cpu_budget)

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "wedges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": {"tip": "tip decomposition (both sides)", "tip_u": "tip decomposition (side U)",
                                "wing": "wing decomposition (all edges)",
                                "batch": "batched tip (side U) and wing decompositions"}[kind] + f" of {g.name}",
                   "graph": graph_cfg, "P": P, "bound_rule": "plain", "m": g_m, "n_u": g.n_u, "n_v": g.n_v},
        "decomposition_ms": round(min(step_ms), 2),
        "phases_ms": phases,
        "work": work,
        "roofline": roofline,
        "copy_kernel": copy,
        "learned_vs_plain": learned,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity or None,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
