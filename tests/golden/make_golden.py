"""Write the oracle's expected results for the full-size seeded workloads.

Calls only ``oracle`` (the CPU oracle) and ``synth`` (the seeded inputs).
For each (workload, quantity) it stores, in ``<workload>__<quantity>.json``:
the SHA-256 of the uint64 result vector (little-endian, entity order), its
length, sum and maximum, and a fixed sample of (index, value) pairs, plus the
oracle's own work counters and wall time.

Usage:  python tests/golden/make_golden.py WORKLOAD QUANTITY [THREADS]
        QUANTITY in {count_u, count_v, count_e, tip_u, tip_v, wing}
        THREADS: host threads for the oracle's counting (default 1; peeling
        is sequential either way, and results do not depend on it)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def sample_idx(n: int, k: int = 64, seed: int = 12345) -> np.ndarray:
    if n == 0:
        return np.zeros(0, np.int64)
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, n, size=min(k, n)))


def main(workload: str, quantity: str, threads: int = 1):
    g = synth.config_graph(workload)
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    stats = {}
    if quantity == "count_u":
        res = oracle.count_vertex(g)[0]
    elif quantity == "count_v":
        res = oracle.count_vertex(g)[1]
    elif quantity == "count_e":
        res = oracle.count_edge(g)
    elif quantity in ("tip_u", "tip_v"):
        res, stats = oracle.tip(g, 0 if quantity == "tip_u" else 1, return_stats=True)
    elif quantity == "wing":
        res, stats = oracle.wing(g, return_stats=True)
    else:
        raise SystemExit(f"unknown quantity {quantity}")
    dt = time.perf_counter() - t0
    idx = sample_idx(res.size)
    rec = dict(
        workload=workload,
        quantity=quantity,
        graph_sha256=g.digest(),
        n=int(res.size),
        sha256=digest(res),
        sum=str(int(res.astype(object).sum())) if res.size else "0",
        max=str(int(res.max())) if res.size else "0",
        sample=[[int(i), str(int(res[i]))] for i in idx],
        oracle_seconds=round(dt, 3),
        oracle_count_threads=threads,
        oracle_stats={k: v for k, v in stats.items() if k != "seconds"},
    )
    path = os.path.join(HERE, f"{workload}__{quantity}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(path, rec["oracle_seconds"], "s")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 1)
