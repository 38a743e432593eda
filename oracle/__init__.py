"""CPU oracle for exact target-set betweenness (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the bench's ``cpu_baseline`` leg may
import this package. The GPU library never loads it and shares no code with it.

``oracle_bc.c`` holds the plain single-threaded target-set Brandes of Sec. 3 (eqs.
parentsall, brandes, centrality) and the restricted search Dijkstra_SK of Sec. 4 (eq.
frontierparents). This module compiles it with gcc and wraps it for numpy arrays, and
adds the plain definitions of the skeleton (Sec. 4: frontiers, the cut edges R, the
clique tuples <d, sigma>, the per-part tables of Sec. 5 Step 3) on top of Dijkstra_SK.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle_bc.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, INVAL, OVERFLOW, NOMEM = 0, 1, 2, 3
ORDERED = 1


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build(out: str = LIB, src: str = SRC) -> str:
    """Compile the oracle with gcc (-O2, no -ffast-math: IEEE rounding is kept)."""
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def lib(path: str | None = None):
    """Load the compiled oracle, building it first only if it is missing."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def _bind(L):
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    L.oracle_sssp.argtypes = [i32, P, P, P, i32, P, P]
    L.oracle_sssp.restype = ctypes.c_int
    L.oracle_dijkstra_sk.argtypes = [i32, P, P, P, P, P, i32, P, P]
    L.oracle_dijkstra_sk.restype = ctypes.c_int
    L.oracle_bc.argtypes = [i32, P, P, P, i32, P, ctypes.c_uint32, P]
    L.oracle_bc.restype = ctypes.c_int
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, np.int64)
    col = np.ascontiguousarray(g.col, np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, np.int32)
    return rp, col, w


def bc(g, S, ordered: bool = False, L=None) -> np.ndarray:
    """Exact betweenness w.r.t. target set S (unordered pairs unless `ordered`)."""
    L = L or lib()
    rp, col, w = _csr(g)
    S = np.ascontiguousarray(S, np.int32)
    out = np.zeros(g.n, np.float64)
    rc = L.oracle_bc(g.n, _ptr(rp), _ptr(col), _ptr(w), S.size, _ptr(S),
                     ORDERED if ordered else 0, _ptr(out))
    if rc:
        raise OracleError(rc, "oracle_bc")
    return out


def sssp(g, s: int, L=None):
    """(d int64 with -1 = unreachable, sigma uint64 with 0 = unreachable) from s."""
    L = L or lib()
    rp, col, w = _csr(g)
    d = np.empty(g.n, np.int64)
    sig = np.empty(g.n, np.uint64)
    rc = L.oracle_sssp(g.n, _ptr(rp), _ptr(col), _ptr(w), int(s), _ptr(d), _ptr(sig))
    if rc:
        raise OracleError(rc, "oracle_sssp")
    return d, sig


def dijkstra_sk(g, label, frontier, f: int, L=None):
    """Dijkstra_SK from frontier f inside its part of `label` (eq. frontierparents)."""
    L = L or lib()
    rp, col, w = _csr(g)
    label = np.ascontiguousarray(label, np.int32)
    frontier = np.ascontiguousarray(frontier, np.uint8)
    d = np.empty(g.n, np.int64)
    sig = np.empty(g.n, np.uint64)
    rc = L.oracle_dijkstra_sk(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(label),
                              _ptr(frontier), int(f), _ptr(d), _ptr(sig))
    if rc:
        raise OracleError(rc, "oracle_dijkstra_sk")
    return d, sig


# ------------------------------------------------------------- the skeleton ----

def prime_labels(n: int, part, k: int, S) -> np.ndarray:
    """Partition P' of Sec. 5 (Step 1, "Target nodes in the skeleton"): every target is
    taken out of its part and becomes a singleton part; the i-th target of S gets label
    k + i."""
    lab = np.asarray(part, np.int64).copy()
    S = np.asarray(S, np.int64)
    lab[S] = k + np.arange(S.size)
    return lab.astype(np.int32)


def frontier_flags(g, label) -> np.ndarray:
    """F_i (Sec. 4, "Nodes in the skeleton"): nodes with an edge to another part."""
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    cross = label[src] != label[g.col]
    fr = np.zeros(g.n, np.uint8)
    fr[src[cross]] = 1
    return fr


def skeleton(g, part, k: int, S, L=None) -> dict:
    """The skeleton of Sec. 4 for partition P', with zero-multiplicity entries pruned.

    Returns a dict:
      nodes     sorted original ids of V_SK (all frontier nodes)
      R         {(u, v): w} cut arcs, both directions
      clique    {(f, q): (d(f,q), sigma(f,q))} for f != q in the same part, sigma > 0
      tables    {v: {f: (d(f,v), sigma(f,v))}} for every non-frontier v, sigma > 0
    """
    L = L or lib()
    lab = prime_labels(g.n, part, k, S)
    fr = frontier_flags(g, lab)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    w = g.w if g.w is not None else np.ones(g.col.size, np.int32)
    R = {}
    for e in np.nonzero(lab[src] != lab[g.col])[0]:
        R[(int(src[e]), int(g.col[e]))] = int(w[e])
    clique = {}
    tables = {}
    for f in np.nonzero(fr)[0]:
        f = int(f)
        d, sig = dijkstra_sk(g, lab, fr, f, L)
        same = np.nonzero((lab == lab[f]) & (sig > 0))[0]
        for v in same:
            v = int(v)
            if v == f:
                continue
            if fr[v]:
                clique[(f, v)] = (int(d[v]), int(sig[v]))
            else:
                tables.setdefault(v, {})[f] = (int(d[v]), int(sig[v]))
    return {
        "nodes": np.nonzero(fr)[0].astype(np.int64),
        "labels": lab,
        "frontier": fr,
        "R": R,
        "clique": clique,
        "tables": tables,
    }
