"""Exhaustive enumeration for tiny graphs (test infrastructure only).

These follow the definitions directly, with no peeling at all:

* a butterfly is a 4-tuple u < u', v < v' with all four edges present
  (Section 2.1);
* the tip number of u is the largest k such that some set S of U-vertices
  containing u has every x in S in at least k butterflies of G[S u V]
  (Definition 2 without its connectivity and maximality clauses, which do not
  change the numbers);
* the wing number of e is the largest k such that some edge set F containing
  e has every f in F in at least k butterflies whose four edges are all in F
  (Definition 1, same remark).

A vertex or edge in no butterfly therefore has entity number 0.
"""
from __future__ import annotations

import itertools

import numpy as np


def _adj(g):
    a = np.zeros((g.n_u, g.n_v), dtype=bool)
    u, v = g.edges()
    a[u, v] = True
    return a


def butterflies(g):
    """All butterflies as (u, u', v, v') with u < u', v < v'."""
    a = _adj(g)
    out = []
    for u, up in itertools.combinations(range(g.n_u), 2):
        common = np.flatnonzero(a[u] & a[up])
        for v, vp in itertools.combinations(common.tolist(), 2):
            out.append((u, up, v, vp))
    return out


def count_vertex(g):
    bu = np.zeros(g.n_u, np.uint64)
    bv = np.zeros(g.n_v, np.uint64)
    for u, up, v, vp in butterflies(g):
        bu[u] += 1
        bu[up] += 1
        bv[v] += 1
        bv[vp] += 1
    return bu, bv


def _edge_id(g):
    eid = {}
    u, v = g.edges()
    for e, (a, b) in enumerate(zip(u.tolist(), v.tolist())):
        eid[(a, b)] = e
    return eid


def _butterfly_edges(g):
    eid = _edge_id(g)
    return [(eid[(u, v)], eid[(u, vp)], eid[(up, v)], eid[(up, vp)]) for u, up, v, vp in butterflies(g)]


def count_edge(g):
    be = np.zeros(g.m, np.uint64)
    for quad in _butterfly_edges(g):
        for e in quad:
            be[e] += 1
    return be


def tip(g, side: int = 0):
    """Max-min over all subsets S of the peeled side (2^n subsets, n <= 14)."""
    n = g.n_u if side == 0 else g.n_v
    if n > 14:
        raise ValueError("brute-force tip is limited to 14 peeled vertices")
    # each butterfly contributes to two vertices of the peeled side
    pairs = [(u, up) if side == 0 else (v, vp) for u, up, v, vp in butterflies(g)]
    theta = np.zeros(n, np.uint64)
    for mask in range(1, 1 << n):
        sup = np.zeros(n, np.int64)
        for a, b in pairs:
            if (mask >> a) & 1 and (mask >> b) & 1:
                sup[a] += 1
                sup[b] += 1
        members = [x for x in range(n) if (mask >> x) & 1]
        k = min(sup[x] for x in members)
        for x in members:
            if k > theta[x]:
                theta[x] = k
    return theta


def wing(g):
    """Max-min over all edge subsets F (2^m subsets, m <= 16)."""
    m = g.m
    if m > 16:
        raise ValueError("brute-force wing is limited to 16 edges")
    quads = _butterfly_edges(g)
    qmask = np.array([sum(1 << e for e in q) for q in quads], dtype=np.int64)
    qedges = np.array(quads, dtype=np.int64).reshape(-1, 4)
    theta = np.zeros(m, np.uint64)
    for mask in range(1, 1 << m):
        inside = (qmask & mask) == qmask
        sup = np.zeros(m, np.int64)
        if inside.any():
            np.add.at(sup, qedges[inside].ravel(), 1)
        members = [e for e in range(m) if (mask >> e) & 1]
        k = min(sup[e] for e in members)
        for e in members:
            if k > theta[e]:
                theta[e] = k
    return theta


def _connected(items, links):
    """True when items (a set) form one component under links (pairs)."""
    items = set(items)
    if len(items) <= 1:
        return True
    adj = {x: set() for x in items}
    for a, b in links:
        if a in items and b in items:
            adj[a].add(b)
            adj[b].add(a)
    start = next(iter(items))
    seen, stack = {start}, [start]
    while stack:
        x = stack.pop()
        for y in adj[x] - seen:
            seen.add(y)
            stack.append(y)
    return seen == items


def _maximal_labels(n, good_sets):
    """Label each element with the smallest id of the maximal good set that
    holds it (-1 if none); the maximal sets must be disjoint."""
    maximal = [s for s in good_sets if not any(s < t for t in good_sets)]
    lab = np.full(n, -1, np.int64)
    for s in maximal:
        for x in s:
            assert lab[x] == -1, "maximal k-sets overlap"
            lab[x] = min(s)
    return lab


def tip_components(g, side: int, k: int):
    """k-tips by Definition 2 read literally: the maximal sets S of the side's
    vertices (with all of the other side) in which every vertex has at least k
    butterflies of G[S u other side] and any two are joined by a chain of
    butterflies; each vertex gets the smallest id of its k-tip, -1 if none."""
    n = g.n_u if side == 0 else g.n_v
    if n > 14:
        raise ValueError("brute-force k-tips are limited to 14 vertices")
    pairs = [(u, up) if side == 0 else (v, vp) for u, up, v, vp in butterflies(g)]
    good = []
    for mask in range(1, 1 << n):
        members = {x for x in range(n) if (mask >> x) & 1}
        inside = [(a, b) for a, b in pairs if a in members and b in members]
        sup = {x: 0 for x in members}
        for a, b in inside:
            sup[a] += 1
            sup[b] += 1
        if min(sup.values()) >= k and _connected(members, inside):
            good.append(frozenset(members))
    return _maximal_labels(n, good)


def wing_components(g, k: int):
    """k-wings by Definition 1 read literally: the maximal edge sets F in
    which every edge lies in at least k butterflies whose four edges are in F
    and any two edges are joined by a chain of such butterflies; each edge
    gets the smallest id of its k-wing, -1 if none."""
    m = g.m
    if m > 16:
        raise ValueError("brute-force k-wings are limited to 16 edges")
    quads = _butterfly_edges(g)
    good = []
    for mask in range(1, 1 << m):
        members = {e for e in range(m) if (mask >> e) & 1}
        inside = [q for q in quads if all(e in members for e in q)]
        sup = {e: 0 for e in members}
        links = []
        for q in inside:
            for e in q:
                sup[e] += 1
            links += [(q[0], q[1]), (q[0], q[2]), (q[0], q[3])]
        if min(sup.values()) >= k and _connected(members, links):
            good.append(frozenset(members))
    return _maximal_labels(m, good)
