"""Brute-force betweenness for tiny graphs, in exact rational arithmetic.

Test infrastructure only (see the package docstring). Two independent routes to the
same definitions, used to pin the C oracle:

* ``floyd_warshall_counts``: all-pairs distances d(s,t) and shortest-path counts
  sigma(s,t) by Floyd-Warshall with path counting. Then the naive algorithm of Sec. 3:
  v lies on a shortest s-t path iff d(s,t) = d(s,v) + d(v,t), in which case
  sigma(s,t|v) = sigma(s,v) * sigma(v,t), and delta(s,t|v) = sigma(s,t|v)/sigma(s,t).
  C(v) sums delta(s,t|v) over target pairs (eq. centrality).
* ``enumerate_shortest_paths``: explicit depth-first enumeration of every simple path,
  keeping those of minimum length; the counts fall out of the path lists.

Both use Python integers (no overflow) and ``fractions.Fraction``.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

INF = None


def adjacency(g):
    adj = [dict() for _ in range(g.n)]
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            v = int(g.col[e])
            adj[u][v] = 1 if g.w is None else int(g.w[e])
    return adj


def floyd_warshall_counts(g):
    """(d, c): d[i][j] int or None (unreachable), c[i][j] the number of shortest paths."""
    n = g.n
    adj = adjacency(g)
    d = [[None] * n for _ in range(n)]
    c = [[0] * n for _ in range(n)]
    for i in range(n):
        d[i][i] = 0
        c[i][i] = 1
        for j, w in adj[i].items():
            d[i][j] = w
            c[i][j] = 1
    for k in range(n):
        for i in range(n):
            dik = d[i][k]
            if dik is None or i == k:
                continue
            for j in range(n):
                if j == k or j == i:
                    continue
                dkj = d[k][j]
                if dkj is None:
                    continue
                alt = dik + dkj
                if d[i][j] is None or alt < d[i][j]:
                    d[i][j] = alt
                    c[i][j] = c[i][k] * c[k][j]
                elif alt == d[i][j]:
                    c[i][j] += c[i][k] * c[k][j]
    return d, c


def bc_from_counts(n, d, c, S, ordered=False):
    """C(v) = sum over target pairs s != t of delta(s,t|v), v not an endpoint."""
    S = [int(s) for s in S]
    C = [Fraction(0)] * n
    for a in range(len(S)):
        for b in range(len(S)):
            if a == b or (not ordered and b < a):
                continue
            s, t = S[a], S[b]
            if d[s][t] is None:
                continue
            for v in range(n):
                if v == s or v == t or d[s][v] is None or d[v][t] is None:
                    continue
                if d[s][v] + d[v][t] == d[s][t]:
                    C[v] += Fraction(c[s][v] * c[v][t], c[s][t])
    return C


def bc_bruteforce(g, S, ordered=False):
    d, c = floyd_warshall_counts(g)
    return bc_from_counts(g.n, d, c, S, ordered)


def enumerate_shortest_paths(g, s, t, allowed=None):
    """All minimum-length simple s-t paths whose nodes pass `allowed(v)` (endpoints are
    always allowed), as (length, [paths])."""
    adj = adjacency(g)
    best = [None]
    found = []

    def rec(v, length, path, seen):
        if best[0] is not None and length > best[0]:
            return
        if v == t:
            if best[0] is None or length < best[0]:
                best[0] = length
                found.clear()
            found.append(list(path))
            return
        for u, w in adj[v].items():
            if u in seen:
                continue
            if u != t and allowed is not None and not allowed(u):
                continue
            seen.add(u)
            path.append(u)
            rec(u, length + w, path, seen)
            path.pop()
            seen.discard(u)

    rec(s, 0, [s], {s})
    return best[0], found


def bc_by_enumeration(g, S, ordered=False):
    """Betweenness from explicit path lists: each shortest s-t path adds
    1/sigma(s,t) to every inner node."""
    S = [int(s) for s in S]
    C = [Fraction(0)] * g.n
    for a in range(len(S)):
        for b in range(len(S)):
            if a == b or (not ordered and b < a):
                continue
            length, paths = enumerate_shortest_paths(g, S[a], S[b])
            if length is None:
                continue
            for p in paths:
                for v in p[1:-1]:
                    C[v] += Fraction(1, len(paths))
    return C


def restricted_counts(g, label, frontier, f):
    """Dijkstra_SK by enumeration: inside the part of f, the G_i distance to every v and
    the number of G_i-shortest f-v paths whose inner nodes are all non-frontier."""
    n = g.n
    part = [v for v in range(n) if label[v] == label[f]]
    sub_adj = adjacency(g)
    inside = set(part)
    out = {}
    for v in part:
        # unrestricted G_i distance
        dist = _dijkstra_plain(sub_adj, f, inside)
        if dist.get(v) is None:
            out[v] = (None, 0)
            continue
        # enumerate paths inside G_i of exactly that length, inner nodes non-frontier
        cnt = _count_paths(sub_adj, f, v, dist[v], inside,
                           lambda u: frontier[u] == 0)
        out[v] = (dist[v], cnt)
    return out


def _dijkstra_plain(adj, s, inside):
    import heapq

    dist = {s: 0}
    pq = [(0, s)]
    while pq:
        dv, v = heapq.heappop(pq)
        if dv != dist[v]:
            continue
        for u, w in adj[v].items():
            if u not in inside:
                continue
            nd = dv + w
            if u not in dist or nd < dist[u]:
                dist[u] = nd
                heapq.heappush(pq, (nd, u))
    return dist


def _count_paths(adj, s, t, length, inside, inner_ok):
    if s == t:
        return 1
    cnt = 0

    def rec(v, rem, seen):
        nonlocal cnt
        for u, w in adj[v].items():
            if u not in inside or u in seen or w > rem:
                continue
            if u == t:
                if w == rem:
                    cnt += 1
                continue
            if not inner_ok(u):
                continue
            seen.add(u)
            rec(u, rem - w, seen)
            seen.discard(u)

    rec(s, length, {s})
    return cnt


def to_float(C):
    return np.array([float(x) for x in C], np.float64)
