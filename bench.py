#!/usr/bin/env python3
"""Benchmark of the MI355X butterfly-peeling path.

Default workload: tip decomposition of side U of the seeded Chung-Lu graph
|U|=5M, |V|=1M, 100M edges, exponent 2.0, degree cap 50k, P=150 -- the
held-out graph on which learned and plain range bounds are compared -- under
the paper's range-bound rule.  A step is one call: preprocessing, priority
counting, coarse-grained peel rounds (replayed from a captured HIP graph,
with recounts) and the fine-grained persistent kernel, all on the GPU with the
graph resident in HBM before the timed region.

Prints one JSON line: wedges/s over the timed steps (value), the per-step
decomposition time, the bound rules compared on the same graph (the paper's
rule, the library's plain rule, learned, learned with perfect predictions),
the roofline of the dominant
kernel class (algorithmic bytes / its HIP-event time on the library's stream,
from a kernel-timing pass), the 20M-edge tip and 5M-edge wing workloads as
extra keys, and the CPU oracle timed on a bounded sample.

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
CLASS_KERNEL = {"tip_hrange": "k_tip_peel_hrange<13, 512>", "tip_tiled": "k_tip_peel_tiled<16, true>",
                "fd": "k_tip_fd / k_wing_fd", "dense": "m_gram", "wing_cd": "w_links / w_blooms"}

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
    "batch_mixed_4096": ("mixed_4096", "batch", 0),
}
# batch lists: (number of graphs, smallest and largest edge count)
BATCHES = {"mixed_1024": (1024, 1e3, 1e5), "mixed_4096": (4096, 1e3, 1e6)}


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


def run_step(pb, ctx, dg, kind, P, flags, rule=0, tune=None):
    """One pass of the hot path; returns (outputs, list of stats dicts)."""
    opts = pb.make_opts(P=P, flags=flags, bound_rule=rule, **(tune or {}))
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


def host_info():
    """Host core count and CPU model of the machine the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), cpu_model=model)


def cpu_baseline(graph_cfg, kind, budget_s):
    """The oracle on a bounded sample: the same generator family scaled down
    until one run takes about budget_s seconds on one host core.  The
    oracle's counting walks exactly the wedges its peeling walks (every
    u -> v -> u' with u' != u, peeled u' included), so a tip run's work is
    twice its peel counter."""
    import oracle
    import synth

    oracle.set_threads(1)
    info = host_info()
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
                           f"{wedges} wedges in {dt:.2f} s", seconds=round(dt, 2), **info)
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
            wedges = 2 * st["wedges"]
        else:
            _, st = oracle.wing(g, return_stats=True)
            wedges = st["wedges"]
        dt = time.perf_counter() - t0
        best = dict(value=wedges / dt if dt > 0 else 0.0, unit="wedges/s", cores=1, kind="oracle",
                    sample=f"{g.name}: {kind} side U by sequential bottom-up peeling, {wedges} wedges in {dt:.2f} s "
                           f"(workload scaled 1/{scale})", seconds=round(dt, 2), **info)
        if dt * 4 > budget_s or scale == 1:
            break
        scale //= 2
    # the oracle's own full-size runs that wrote the stored results
    full = []
    for wl, q in (("cl_5m_1m_100m", "tip_u"), ("cl_1m_200k_20m", "tip_u"), ("cl_1m_200k_20m", "tip_v"),
                  ("cl_500k_100k_5m", "wing")):
        rec = golden(wl, q)
        if rec:
            w = rec.get("oracle_stats", {}).get("wedges")
            full.append(dict(workload=wl, quantity=q, oracle_seconds=rec["oracle_seconds"],
                             count_threads=rec.get("oracle_count_threads", 1), peel_wedges=w))
    best["full_size_oracle_runs"] = full
    return best


def load_graph(graph_cfg, cache_dir, synth):
    """The seeded graph, from an .npz cache when one is given and present."""
    if cache_dir:
        path = os.path.join(cache_dir, f"{graph_cfg}.npz")
        if os.path.exists(path):
            z = np.load(path)
            g = synth.Graph(int(z["n_u"]), int(z["n_v"]), z["row_ptr"], z["col_idx"], str(z["name"]))
            log(f"[bench] loaded {graph_cfg} from {path}")
            return g
    g = synth.config_graph(graph_cfg, log=log)
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(os.path.join(cache_dir, f"{graph_cfg}.npz"), row_ptr=g.row_ptr, col_idx=g.col_idx, n_u=g.n_u,
                 n_v=g.n_v, name=g.name)
    return g


def side_entry(pb, st, q, res, graph_cfg, ref=None):
    rec = golden(graph_cfg, q)
    imb = st["fd_work_max"] / max(st["fd_work_sum"] / max(st["partitions"], 1), 1)
    d = dict(side=q, ms_total=round(st["ms_total"], 2), ms_cd=round(st["ms_cd"], 2), ms_fd=round(st["ms_fd"], 2),
             rho=st["rho"], partitions=st["partitions"], fd_imbalance=round(imb, 2), rule_used=st["bound_rule_used"],
             exact=(digest(pb.to_numpy_u64(res)) == rec["sha256"]) if rec else None)
    if ref is not None:
        d["identical_to_paper_rule"] = digest(pb.to_numpy_u64(res)) == ref
    return d


def extra_workload(pb, torch, ctx, name, cache_dir):
    """One warm and one measured pass of another workload (time and parity)."""
    import synth

    graph_cfg, kind, P = WORKLOADS[name]
    g = load_graph(graph_cfg, cache_dir, synth)
    dg = pb.DeviceGraph.from_graph(g)
    run_step(pb, ctx, dg, kind, P, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, stats = run_step(pb, ctx, dg, kind, P, 0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    qn = {"tip": ["tip_u", "tip_v"], "tip_u": ["tip_u"], "wing": ["wing"]}[kind]
    parity = {}
    for q, t in zip(qn, outs):
        rec = golden(graph_cfg, q)
        parity[q] = (digest(pb.to_numpy_u64(t)) == rec["sha256"]) if rec else None
    wedges = sum(s["wedges"] for s in stats)
    d = dict(workload=g.name, ms=round(ms, 2), wedges=wedges, wedges_per_s=round(wedges / (ms / 1e3), 1),
             phases_ms=[{k: round(s[k], 2) for k in ("ms_total", "ms_count", "ms_cd", "ms_fd_prep", "ms_fd")}
                        for s in stats],
             rho=[s["rho"] for s in stats], bound_rule="plain", parity_vs_oracle=parity)
    if kind == "wing":
        d.update(updates=stats[0]["updates"], links=stats[0]["links"], blooms=stats[0]["blooms"])
    # the paper's ablations (Section 6, Figs 6 and 9): PBNG- keeps peeled
    # entities in the lists (no dynamic graph updates); PBNG-- also drops
    # batching (tip: never recounts; wing: every peeled edge walks its blooms
    # instead of one aggregated update per bloom)
    abl = {"PBNG": dict(ms=round(ms, 2), wedges=wedges, updates=sum(s["updates"] for s in stats))}
    variants = [("PBNG-", pb.F_NO_DYNAMIC), ("PBNG--", pb.F_NO_DYNAMIC | pb.F_NO_BATCH)]
    for vname, fl in variants:
        t0 = time.perf_counter()
        outs_v, stats_v = run_step(pb, ctx, dg, kind, P, fl)
        torch.cuda.synchronize()
        vms = (time.perf_counter() - t0) * 1e3
        same = all(digest(pb.to_numpy_u64(a)) == digest(pb.to_numpy_u64(b)) for a, b in zip(outs, outs_v))
        abl[vname] = dict(ms=round(vms, 2), wedges=sum(s["wedges"] for s in stats_v),
                          updates=sum(s["updates"] for s in stats_v), identical=same)
    d["ablation"] = abl
    del dg
    return d


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tip_u_cl_5m_1m_100m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the comparison of bound rules")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads' extra keys")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--graph-cache", default=None, help="directory for .npz copies of the generated graphs")
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
        graphs = synth.mixed_graphs(range(nb), m_min, m_max)
        g = synth.Graph(n_u=sum(x.n_u for x in graphs), n_v=sum(x.n_v for x in graphs),
                        row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
                        name=f"{nb} graphs, m log-uniform in [{m_min:.0e}, {m_max:.0e}], half ER half CL")
        g_m = sum(x.m for x in graphs)
    else:
        g = load_graph(graph_cfg, args.graph_cache, synth)
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

    # single graphs: the paper's bound rule (Section 3.1.3; the other rules
    # are compared below).  Batches: learned bounds (when a predictor is
    # stored) and the autotuner's hub cut-over and key-tile threshold, tuned
    # on the largest graph.
    rule, tune, tuned = (pb.BOUND_PAPER if kind in ("tip", "tip_u") else 0), None, None
    if kind == "batch":
        from paper_2110_12511_amd import predictor

        if predictor.install(ctx):
            rule = pb.BOUND_LEARNED
        big = max(range(len(graphs)), key=lambda i: graphs[i].m)
        bt, bms = ctx.autotune(dg[big], 0)
        bw, wms = ctx.autotune(dg[big], 2)
        tune = dict(dense_cut=bt.dense_cut, tile_w=bt.tile_w)
        tuned = dict(graph=graphs[big].name,
                     tip=dict(dense_cut=bt.dense_cut, tile_w=bt.tile_w, recount_w=bt.recount_w, P=bt.P,
                              ms=round(bms, 2)),
                     wing=dict(dense_cut=bw.dense_cut, wide_work=bw.wide_work, P=bw.P, ms=round(wms, 2)))
        log(f"[bench] autotuned on {graphs[big].name}: {tuned}")

    for i in range(args.warmup):
        run_step(pb, ctx, dg, kind, P, 0, rule, tune)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")

    # timed steps: the library's default path (captured coarse-grained rounds)
    step_ms, all_stats, outs = [], [], None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        outs, stats = run_step(pb, ctx, dg, kind, P, 0, rule, tune)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        all_stats.append(stats)
        log(f"[bench] step {i + 1}/{args.steps}: {step_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_all

    wedges_per_step = [sum(s["wedges"] for s in st) for st in all_stats]
    value = sum(wedges_per_step) / total_s
    ms_per_step = total_s * 1e3 / args.steps

    # kernel-timing pass: HIP events around every kernel class on the
    # library's stream (coarse-grained tip rounds are host-driven under
    # timing, since events recorded inside a captured graph cannot be timed;
    # the kernels and their grids of work are the same)
    _, tstats = run_step(pb, ctx, dg, kind, P, pb.binding.F_KERNEL_TIMING, rule, tune)
    torch.cuda.synchronize()
    agg = {}
    for s in tstats:
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
                    kernel_wedges_per_s=round(d["wedges"] / (d["ms"] / 1e3), 1) if d["ms"] > 0 else 0.0,
                    timing_pass_ms=round(sum(s["ms_total"] for s in tstats), 2),
                    classes_ms={n: round(a["ms"], 2) for n, a in agg.items() if a["ms"] > 0})

    # parity evidence against stored oracle results (when present)
    parity = {}
    qnames = {"tip": ["tip_u", "tip_v"], "tip_u": ["tip_u"], "wing": ["wing"]}.get(kind, [])
    for q, t in zip(qnames, outs):
        rec = golden(graph_cfg, q)
        if rec is not None:
            parity[q] = digest(pb.to_numpy_u64(t)) == rec["sha256"]
    if kind == "batch":
        rec = golden(graph_cfg, "batch")
        if rec is not None:
            ent = rec["entries"]
            for q, res in (("tip_u", outs[0]), ("wing", outs[1])):
                ok, n = 0, 0
                for i, (x, t) in enumerate(zip(graphs, res)):
                    e = ent[str(i)]
                    if q in e:
                        n += 1
                        ok += int(e["graph"] == x.digest()[:16] and digest(pb.to_numpy_u64(t))[:16] == e[q])
                parity[q] = dict(graphs_checked=n, graphs_identical=ok, of=len(graphs))

    last = all_stats[-1]
    phases = [{k: round(s[k], 2) for k in ("ms_total", "ms_prep", "ms_count", "ms_cd", "ms_fd_prep", "ms_fd")}
              for s in last]
    work = [{k: s[k] for k in ("wedges", "wedges_count", "wedges_cd", "wedges_fd", "rho", "recounts", "partitions",
                                "P_used", "fd_work_max", "fd_work_sum", "updates", "links", "blooms")} for s in last]

    # bound rules on the same graph and P, outside the timed steps (tip
    # workloads): the paper's rule, the library's plain rule, learned
    rules = None
    if kind in ("tip", "tip_u") and not args.no_learned:
        from paper_2110_12511_amd import predictor

        have_pred = predictor.install(ctx)
        rules = {}
        ref = {}
        for rule_name, rrule in (("paper", pb.BOUND_PAPER), ("plain", pb.BOUND_PLAIN), ("learned", pb.BOUND_LEARNED)):
            if rule_name == "learned" and not have_pred:
                continue
            per_side = []
            for side in ((pb.SIDE_U, pb.SIDE_V) if kind == "tip" else (pb.SIDE_U,)):
                t = pb.tip(ctx, dg, side, pb.make_opts(P=P, bound_rule=rrule))
                torch.cuda.synchronize()
                q = "tip_u" if side == pb.SIDE_U else "tip_v"
                if rule_name == "paper":
                    ref[q] = digest(pb.to_numpy_u64(t))
                per_side.append(side_entry(pb, ctx.stats(), q, t, graph_cfg, ref.get(q) if rule_name != "paper" else None))
            rules[rule_name] = per_side
            log(f"[bench] bound rule {rule_name}: " + ", ".join(f"{e['side']} {e['ms_total']} ms" for e in per_side))
        # the learned rule with perfect predictions (the exact tip numbers as
        # hint): the most any predictor could change the schedule
        per_side = []
        for side in ((pb.SIDE_U, pb.SIDE_V) if kind == "tip" else (pb.SIDE_U,)):
            q = "tip_u" if side == pb.SIDE_U else "tip_v"
            exact = pb.tip(ctx, dg, side, pb.make_opts(P=P, bound_rule=pb.BOUND_PAPER))
            t = pb.tip_hinted(ctx, dg, side, exact, pb.make_opts(P=P))
            torch.cuda.synchronize()
            per_side.append(side_entry(pb, ctx.stats(), q, t, graph_cfg, ref.get(q)))
            del exact
        rules["learned_perfect_predictions"] = per_side
        log("[bench] learned rule, perfect predictions: " + ", ".join(f"{e['side']} {e['ms_total']} ms" for e in per_side))

    extras = None
    if not args.no_extras and args.workload == "tip_u_cl_5m_1m_100m":
        del outs
        extras = {}
        for name in ("tip_cl_1m_200k_20m", "wing_cl_500k_100k_5m"):
            extras[name] = extra_workload(pb, torch, ctx, name, args.graph_cache)
            log(f"[bench] extra {name}: {extras[name]['ms']} ms")

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
                   "graph": graph_cfg, "P": P,
                   "bound_rule": {pb.BOUND_PAPER: "paper", pb.BOUND_LEARNED: "learned"}.get(rule, "plain"), "m": g_m,
                   "n_u": g.n_u, "n_v": g.n_v},
        "decomposition_ms": round(min(step_ms), 2),
        "phases_ms": phases,
        "work": work,
        "roofline": roofline,
        "copy_kernel": copy,
        "bound_rules": rules,
        "extras": extras,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity or None,
    }
    if kind == "batch":
        line["config"].update(graphs=len(graphs), bound_rule="learned" if rule == pb.BOUND_LEARNED else "plain",
                              autotuned=tuned, batch_chunks_edges=2 ** 26)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
