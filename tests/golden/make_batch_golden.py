"""Oracle results for the batch of 4096 graphs of uneven sizes.

Calls only ``oracle`` (the CPU oracle) and ``synth`` (the seeded inputs).
The family is synth.mixed_graph(gi, 1e3, 1e6) for gi = 0 .. 4095: edge
counts log-uniform in [1e3, 1e6], even gi Erdos-Renyi, odd gi Chung-Lu.
Tip numbers of side U are computed for every graph; wing numbers for every
graph with at most WING_MAX_M edges plus a seeded sample of WING_SAMPLE
larger ones (the oracle's wing peeling of a million-edge graph takes minutes).
Each entry stores the first 16 hex digits of the SHA-256 of the graph and of
each result (uint64 little-endian, entity order).

Usage:  python tests/golden/make_batch_golden.py [WORKERS]
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


def plan():
    ms = np.array([synth.mixed_edges(i, M_MIN, M_MAX) for i in range(N_GRAPHS)])
    big = np.flatnonzero(ms > WING_MAX_M)
    rng = np.random.default_rng(4096)
    sample = set(int(i) for i in rng.choice(big, size=min(WING_SAMPLE, big.size), replace=False))
    wing = set(int(i) for i in np.flatnonzero(ms <= WING_MAX_M)) | sample
    return ms, wing, sorted(sample)


def work(args):
    gi, do_wing = args
    g = synth.mixed_graph(gi, M_MIN, M_MAX)
    t0 = time.perf_counter()
    rec = dict(m=g.m, graph=g.digest()[:16], tip_u=sha16(oracle.tip(g, 0)))
    if do_wing:
        rec["wing"] = sha16(oracle.wing(g))
    rec["seconds"] = round(time.perf_counter() - t0, 3)
    return gi, rec


def main(workers: int):
    ms, wing, sample = plan()
    # largest first, so the pool's tail is short
    order = sorted(range(N_GRAPHS), key=lambda i: -int(ms[i]))
    entries = {}
    t0 = time.perf_counter()
    with ProcessPoolExecutor(workers) as ex:
        for k, (gi, rec) in enumerate(ex.map(work, [(i, i in wing) for i in order], chunksize=1)):
            entries[gi] = rec
            if (k + 1) % 256 == 0:
                print(f"{k + 1}/{N_GRAPHS} graphs, {time.perf_counter() - t0:.0f} s", flush=True)
    doc = dict(
        family=f"synth.mixed_graph(gi, {M_MIN:g}, {M_MAX:g}) for gi in 0..{N_GRAPHS - 1}",
        n_graphs=N_GRAPHS,
        edges_total=int(ms.sum()),
        tip_u_covered=N_GRAPHS,
        wing_covered=len(wing),
        wing_rule=f"every graph with m <= {WING_MAX_M}, plus the seeded sample {sample}",
        oracle_cpu_seconds=round(sum(r["seconds"] for r in entries.values()), 1),
        wall_seconds=round(time.perf_counter() - t0, 1),
        workers=workers,
        entries={str(i): entries[i] for i in range(N_GRAPHS)},
    )
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(OUT, doc["wall_seconds"], "s", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4)
