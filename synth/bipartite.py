"""Seeded bipartite graph generators (inputs only; no decomposition logic)."""
from __future__ import annotations

import dataclasses
import hashlib
import os

import numpy as np


@dataclasses.dataclass
class Graph:
    """U-side CSR of a simple bipartite graph.

    row_ptr: int64[n_u+1], row_ptr[0] == 0, row_ptr[n_u] == m
    col_idx: int32[m], V ids in [0, n_v), strictly increasing in each row
    """

    n_u: int
    n_v: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col_idx.shape[0])

    def edges(self):
        """(u, v) int64 arrays in edge-id order."""
        u = np.repeat(np.arange(self.n_u, dtype=np.int64), np.diff(self.row_ptr))
        return u, self.col_idx.astype(np.int64)

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.array([self.n_u, self.n_v, self.m], dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col_idx, dtype=np.int32).tobytes())
        return h.hexdigest()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


def _from_keys(keys: np.ndarray, n_u: int, n_v: int, name: str) -> Graph:
    keys = np.sort(keys.astype(np.int64))
    u = keys // n_v
    v = (keys % n_v).astype(np.int32)
    counts = np.bincount(u, minlength=n_u).astype(np.int64)
    row_ptr = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n_u, n_v, row_ptr, v, name)


def from_edges(n_u: int, n_v: int, edges, name: str = "") -> Graph:
    """Build a Graph from an iterable of distinct (u, v) pairs."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size and (e[:, 0].min() < 0 or e[:, 0].max() >= n_u or e[:, 1].min() < 0 or e[:, 1].max() >= n_v):
        raise ValueError("edge endpoint out of range")
    keys = e[:, 0] * n_v + e[:, 1]
    if np.unique(keys).size != keys.size:
        raise ValueError("duplicate edge")
    return _from_keys(keys, n_u, n_v, name)


def _first_distinct(draws: list, m: int) -> np.ndarray:
    """The first m distinct values of the concatenated draws, in draw order."""
    allk = np.concatenate(draws)
    uniq, first = np.unique(allk, return_index=True)
    if uniq.size < m:
        return None
    order = np.argsort(first, kind="stable")[:m]
    return uniq[order]


def er(n_u: int, n_v: int, m: int, seed: int) -> Graph:
    """m distinct (u, v) pairs uniform over U x V."""
    total = n_u * n_v
    if m > total:
        raise ValueError("m exceeds |U||V|")
    rng = _rng(seed)
    draws = []
    batch = max(1024, int(m * 1.1) + 16)
    while True:
        draws.append(rng.integers(0, total, size=batch, dtype=np.int64))
        keys = _first_distinct(draws, m)
        if keys is not None:
            break
        batch = max(1024, m // 4)
    return _from_keys(keys, n_u, n_v, f"ER({n_u},{n_v},{m},seed={seed})")


def _capped_weights(n: int, m: int, gamma: float, cap: float) -> np.ndarray:
    r = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    if cap * n < m:
        raise ValueError("cap too small for m")
    lo, hi = 0.0, float(m) / r[-1] * 2.0 + 1.0
    for _ in range(200):
        c = 0.5 * (lo + hi)
        s = np.minimum(c * r, cap).sum()
        if s < m:
            lo = c
        else:
            hi = c
    return np.minimum(hi * r, cap)


def _searchsorted_right(cdf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """np.searchsorted(cdf, x, side="right"), element by element, on several
    host threads for large x (numpy releases the interpreter lock inside)."""
    n = x.shape[0]
    if n < (1 << 22):
        return np.searchsorted(cdf, x, side="right")
    from concurrent.futures import ThreadPoolExecutor

    out = np.empty(n, dtype=np.int64)
    k = min(16, os.cpu_count() or 1)
    bounds = np.linspace(0, n, k + 1).astype(np.int64)

    def part(i):
        a, b = bounds[i], bounds[i + 1]
        out[a:b] = np.searchsorted(cdf, x[a:b], side="right")

    with ThreadPoolExecutor(k) as ex:
        list(ex.map(part, range(k)))
    return out


def chung_lu(n_u: int, n_v: int, m: int, gamma: float, cap: float, seed: int, log=None) -> Graph:
    """Chung-Lu bipartite graph with power-law expected degrees on both sides.
    ``log`` (optional) receives a progress line after every draw round."""
    rng = _rng(seed)
    wu = _capped_weights(n_u, m, gamma, min(cap, n_v))
    wv = _capped_weights(n_v, m, gamma, min(cap, n_u))
    pu = rng.permutation(n_u).astype(np.int64)
    pv = rng.permutation(n_v).astype(np.int64)
    cu = np.cumsum(wu)
    cu /= cu[-1]
    cv = np.cumsum(wv)
    cv /= cv[-1]
    draws = []
    batch = int(m * 1.25) + 1024
    for _ in range(64):
        xu = _searchsorted_right(cu, rng.random(batch))
        xv = _searchsorted_right(cv, rng.random(batch))
        if log:
            log(f"[synth] CL({n_u},{n_v},{m}): {batch} endpoint pairs drawn")
        np.minimum(xu, n_u - 1, out=xu)
        np.minimum(xv, n_v - 1, out=xv)
        draws.append(pu[xu] * n_v + pv[xv])
        keys = _first_distinct(draws, m)
        if log:
            log(f"[synth] CL({n_u},{n_v},{m}): draw round {_ + 1} done")
        if keys is not None:
            return _from_keys(keys, n_u, n_v, f"CL({n_u},{n_v},{m},g={gamma},cap={cap},seed={seed})")
        # keep the distinct draws only, to bound memory
        allk = np.concatenate(draws)
        uniq, first = np.unique(allk, return_index=True)
        draws = [uniq[np.argsort(first, kind="stable")]]
        batch = max(1024, int((m - uniq.size) * 2.0) + 1024)
    raise RuntimeError("Chung-Lu draw did not reach m distinct edges")


def complete(a: int, b: int) -> Graph:
    keys = (np.arange(a, dtype=np.int64)[:, None] * b + np.arange(b, dtype=np.int64)[None, :]).ravel()
    return _from_keys(keys, a, b, f"K({a},{b})")


def disjoint_union(graphs) -> Graph:
    n_u = sum(g.n_u for g in graphs)
    n_v = sum(g.n_v for g in graphs)
    keys = []
    ou = ov = 0
    for g in graphs:
        u, v = g.edges()
        keys.append((u + ou) * n_v + (v + ov))
        ou += g.n_u
        ov += g.n_v
    return _from_keys(np.concatenate(keys) if keys else np.zeros(0, np.int64), n_u, n_v, "union")


def random_small(n_u: int, n_v: int, p: float, seed: int) -> Graph:
    """Each of the n_u*n_v pairs present independently with probability p."""
    rng = _rng(seed)
    mask = rng.random((n_u, n_v)) < p
    keys = np.flatnonzero(mask.ravel()).astype(np.int64)
    return _from_keys(keys, n_u, n_v, f"G({n_u},{n_v},p={p},seed={seed})")


# Workloads shaped like the paper's bipartite graphs (real datasets are not
# available; these seeded graphs stand in for them).
CONFIGS = {
    "er_2k_1k_20k": dict(kind="er", n_u=2000, n_v=1000, m=20000, seed=1),
    "cl_1m_200k_20m": dict(kind="cl", n_u=1_000_000, n_v=200_000, m=20_000_000, gamma=2.1, cap=50_000, seed=2),
    "cl_500k_100k_5m": dict(kind="cl", n_u=500_000, n_v=100_000, m=5_000_000, gamma=2.3, cap=50_000, seed=3),
    "cl_5m_1m_100m": dict(kind="cl", n_u=5_000_000, n_v=1_000_000, m=100_000_000, gamma=2.0, cap=50_000, seed=4),
}


def _mixed_args(gi: int, m_min: float, m_max: float):
    rng = np.random.default_rng(50000 + gi)
    m = int(round(np.exp(rng.uniform(np.log(m_min), np.log(m_max)))))
    if gi % 2 == 0:
        return ("er", max(m // 10, 2), max(m // 20, 2), m, 0.0)
    return ("cl", max(m // 10, 2), max(m // 50, 2), m, float(rng.uniform(2.0, 2.6)))


def mixed_graph(gi: int, m_min: float = 1e3, m_max: float = 1e6) -> Graph:
    """Graph gi of a family of uneven sizes for batched calls: m log-uniform in
    [m_min, m_max]; even gi Erdos-Renyi with |U| = m/10, |V| = m/20; odd gi
    Chung-Lu with exponent uniform in [2.0, 2.6], |U| = m/10, |V| = m/50,
    degree cap 50000.  Seeds 50000 + gi."""
    kind, n_u, n_v, m, gamma = _mixed_args(gi, m_min, m_max)
    if kind == "er":
        return er(n_u, n_v, m, seed=50000 + gi)
    return chung_lu(n_u, n_v, m, gamma, 50000, seed=50000 + gi)


def mixed_edges(gi: int, m_min: float = 1e3, m_max: float = 1e6) -> int:
    """Edge count of mixed_graph(gi) without drawing the graph."""
    return _mixed_args(gi, m_min, m_max)[3]


def _mixed_worker(args):
    g = mixed_graph(*args)
    return g.n_u, g.n_v, g.row_ptr, g.col_idx, g.name


def mixed_graphs(indices, m_min: float = 1e3, m_max: float = 1e6, workers: int = 0):
    """mixed_graph(gi) for every gi of indices, drawn by a pool of host
    processes (workers = 0: one per core, at most 16); same graphs as one
    at a time."""
    indices = list(indices)
    k = workers or min(16, os.cpu_count() or 1)
    if k <= 1 or len(indices) < 8:
        return [mixed_graph(i, m_min, m_max) for i in indices]
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp

    # fresh interpreters: the caller may hold GPU state that a fork would copy
    with ProcessPoolExecutor(k, mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_mixed_worker, [(i, m_min, m_max) for i in indices], chunksize=4))
    return [Graph(n_u, n_v, rp, ci, name) for n_u, n_v, rp, ci, name in out]


def config_graph(name: str, log=None) -> Graph:
    c = dict(CONFIGS[name])
    kind = c.pop("kind")
    if kind == "er":
        return er(**c)
    return chung_lu(**c, log=log)


