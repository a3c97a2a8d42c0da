"""Oracle results for the batch of 4096 graphs of uneven sizes.

Calls only ``oracle`` (the CPU oracle) and ``synth`` (the seeded inputs).
The family is synth.mixed_graph(gi, 1e3, 1e6) for gi = 0 .. 4095: edge
counts log-uniform in [1e3, 1e6], even gi Erdos-Renyi, odd gi Chung-Lu.
Tip numbers of side U are computed for every graph; wing numbers for every
graph with at most WING_MAX_M edges plus a seeded sample of WING_SAMPLE
larger ones, or, with --wing-all, for every graph.  Each entry stores the
first 16 hex digits of the SHA-256 of the graph and of each result (uint64
little-endian, entity order).  Entries already in the output file whose
graph digest matches are kept, so a run only computes what is missing.

Usage:  python tests/golden/make_batch_golden.py [WORKERS] [--wing-all]
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

N_GRAPHS = 4096
M_MIN, M_MAX = 1e3, 1e6
WING_MAX_M = 300_000
WING_SAMPLE = 8
OUT = os.path.join(HERE, "mixed_4096__batch.json")


def sha16(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()[:16]


def plan(wing_all: bool):
    ms = np.array([synth.mixed_edges(i, M_MIN, M_MAX) for i in range(N_GRAPHS)])
    if wing_all:
        return ms, set(range(N_GRAPHS)), []
    big = np.flatnonzero(ms > WING_MAX_M)
    rng = np.random.default_rng(4096)
    sample = set(int(i) for i in rng.choice(big, size=min(WING_SAMPLE, big.size), replace=False))
    wing = set(int(i) for i in np.flatnonzero(ms <= WING_MAX_M)) | sample
    return ms, wing, sorted(sample)


def work(args):
    gi, do_tip, do_wing, rec = args
    g = synth.mixed_graph(gi, M_MIN, M_MAX)
    rec = dict(rec or {})
    if rec.get("graph") != g.digest()[:16]:
        rec = {}
        do_tip = True
    t0 = time.perf_counter()
    rec.update(m=g.m, graph=g.digest()[:16])
    if do_tip:
        rec["tip_u"] = sha16(oracle.tip(g, 0))
    if do_wing:
        rec["wing"] = sha16(oracle.wing(g))
    rec["seconds"] = round(rec.get("seconds", 0.0) + time.perf_counter() - t0, 3)
    return gi, rec


def main(workers: int, wing_all: bool):
    ms, wing, sample = plan(wing_all)
    old = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            old = {int(k): v for k, v in json.load(f)["entries"].items()}
    # largest first, so the pool's tail is short
    order = sorted(range(N_GRAPHS), key=lambda i: -int(ms[i]))
    jobs = [(i, "tip_u" not in old.get(i, {}), i in wing and "wing" not in old.get(i, {}), old.get(i)) for i in order]
    entries = {}
    t0 = time.perf_counter()
    with ProcessPoolExecutor(workers) as ex:
        for k, (gi, rec) in enumerate(ex.map(work, jobs, chunksize=1)):
            entries[gi] = rec
            if (k + 1) % 256 == 0:
                print(f"{k + 1}/{N_GRAPHS} graphs, {time.perf_counter() - t0:.0f} s", flush=True)
    covered = sum(1 for r in entries.values() if "wing" in r)
    doc = dict(
        family=f"synth.mixed_graph(gi, {M_MIN:g}, {M_MAX:g}) for gi in 0..{N_GRAPHS - 1}",
        n_graphs=N_GRAPHS,
        edges_total=int(ms.sum()),
        tip_u_covered=N_GRAPHS,
        wing_covered=covered,
        wing_rule="every graph" if wing_all else f"every graph with m <= {WING_MAX_M}, plus the seeded sample {sample}",
        oracle_cpu_seconds=round(sum(r["seconds"] for r in entries.values()), 1),
        wall_seconds=round(time.perf_counter() - t0, 1),
        workers=workers,
        entries={str(i): entries[i] for i in range(N_GRAPHS)},
    )
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(OUT, doc["wall_seconds"], "s", flush=True)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    main(int(args[0]) if args else 4, "--wing-all" in sys.argv[1:])
