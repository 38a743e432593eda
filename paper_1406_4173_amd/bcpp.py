"""Python binding of libbcpp.so: argument marshalling only.

Every entry point below forwards to the C function of the same name declared in
include/bcpp.h; all computation happens in the library's HIP kernels. The library must
be built (``python -m paper_1406_4173_amd.build_lib``); if it is missing, loading fails
with an error. There is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcpp.so")

BC_OK, BC_E_INVAL, BC_E_OVERFLOW, BC_E_NOMEM, BC_E_DEVICE, BC_E_AGAIN, BC_E_NOTFOUND = range(7)
BC_ORDERED = 0x1
BC_ENGINE_ONLY = 0x2
BC_NO_GRAPH = 0x4
BC_BATCH_PLAIN = 0x0
BC_BATCH_PP = 0x100
KERNELS = ["select", "settle", "push", "backward", "centrality", "sched", "other", "resident", "dijkstra_sk"]

_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


class BcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bcpp status {code}: {msg}")
        self.code = code


class bc_csr(ctypes.Structure):
    _fields_ = [("n", _i32), ("nnz", _i64), ("row_ptr", _P), ("col", _P), ("w", _P)]


class bc_sk_stats(ctypes.Structure):
    _fields_ = [("n", _i32), ("n_sk", _i32), ("k_prime", _i32), ("largest_part", _i32),
                ("r_arcs", _i64), ("clique_arcs", _i64), ("clique_pruned", _i64),
                ("table_nnz", _i64), ("table_pruned", _i64), ("dsk_sources", _i64),
                ("device_bytes", _i64)]


class bc_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("failed", _i64), ("queued", _i64),
                ("inflight", _i64), ("iterations", _i64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("peak_bytes", _i64), ("cache_bytes", _i64),
                ("dsk_groups_cached", _i64), ("dsk_groups_run", _i64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1406_4173_amd.build_lib")
        # torch ships its own HIP runtime; loading it first makes the library bind to
        # that same runtime (same soname), so torch tensors and streams can be passed in.
        # Loading the library first would put a second HIP runtime in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "bc_last_error": (ctypes.c_char_p, []),
            "bc_graph_create": (ctypes.c_int, [ctypes.POINTER(bc_csr), _P, ctypes.POINTER(_P)]),
            "bc_graph_destroy": (None, [_P]),
            "bc_sssp_counts": (ctypes.c_int, [_P, _P, _i32, _P, _P]),
            "bc_brandes_plain": (ctypes.c_int, [_P, _P, _i32, _u32, _P]),
            "bc_brandes_plain_dev": (ctypes.c_int, [_P, _P, _i32, _u32, _P]),
            "bc_brandes_plain_noalloc": (ctypes.c_int, [_P, _P, _i32, _u32, _P]),
            "bc_noalloc_scratch_bytes": (ctypes.c_size_t, []),
            "bc_partition_sk": (ctypes.c_int, [_P, _P, _i32, _P, _i32, ctypes.POINTER(_P)]),
            "bc_skeleton_destroy": (None, [_P]),
            "bc_skeleton_stats": (ctypes.c_int, [_P, ctypes.POINTER(bc_sk_stats)]),
            "bc_skeleton_export": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
            "bc_skeleton_sssp_counts": (ctypes.c_int, [_P, _P, _i32, _P, _P]),
            "bc_brandes_pp": (ctypes.c_int, [_P, _P, _u32, _P]),
            "bc_brandes_pp_dev": (ctypes.c_int, [_P, _P, _u32, _P]),
            "bc_brandes_pp_all": (ctypes.c_int, [_P, _P, _i32, _u32, _P]),
            "bc_partition_lp": (ctypes.c_int, [_P, _i32, _i32, ctypes.c_uint64, _P, ctypes.POINTER(_i32)]),
            "bc_batch_create": (ctypes.c_int, [_i32, _P, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
            "bc_batch_run": (ctypes.c_int, [_P, _u32, _P]),
            "bc_batch_destroy": (None, [_P]),
            "bc_server_create": (ctypes.c_int, [ctypes.c_size_t, _i32, ctypes.POINTER(_P)]),
            "bc_server_add_graph": (ctypes.c_int, [_P, ctypes.POINTER(bc_csr), _P, _i32,
                                                   ctypes.POINTER(_i32)]),
            "bc_query_submit": (ctypes.c_int, [_P, _i32, _P, _i32, _u32, ctypes.POINTER(_u64)]),
            "bc_query_poll": (ctypes.c_int, [_P, _u64, _P, ctypes.POINTER(_i32)]),
            "bc_server_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(bc_server_stats)]),
            "bc_server_destroy": (None, [_P]),
            "bc_profile_enable": (None, [ctypes.c_int]),
            "bc_profile_read": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64),
                                               ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double)]),
            "bc_profile_reset": (None, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != BC_OK:
        raise BcError(rc, lib().bc_last_error().decode())


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _i32a(x):
    return np.ascontiguousarray(np.asarray(x, np.int32))


def _csr_struct(g):
    rp = np.ascontiguousarray(g.row_ptr, np.int64)
    col = np.ascontiguousarray(g.col, np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, np.int32)
    s = bc_csr(int(g.n), int(rp[-1]) if rp.size else 0, rp.ctypes.data, col.ctypes.data,
               None if w is None else w.ctypes.data)
    return s, (rp, col, w)


class Graph:
    """Device-resident graph handle (bc_graph_create)."""

    def __init__(self, g, stream=None):
        self.n = int(g.n)
        self.m = int(g.row_ptr[-1]) // 2
        s, keep = _csr_struct(g)
        h = _P()
        _check(lib().bc_graph_create(ctypes.byref(s), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.src = g

    def close(self):
        if self.h:
            lib().bc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def sssp_counts(G: Graph, src):
    src = _i32a(src)
    d = np.empty((src.size, G.n), np.int64)
    sig = np.empty((src.size, G.n), np.uint64)
    _check(lib().bc_sssp_counts(G.h, _p(src), src.size, _p(d), _p(sig)))
    return d, sig


def _flags(ordered: bool, engine_only: bool) -> int:
    return (BC_ORDERED if ordered else 0) | (BC_ENGINE_ONLY if engine_only else 0)


def brandes_plain(G: Graph, S, ordered: bool = False, engine_only: bool = False):
    S = _i32a(S)
    out = np.empty(G.n, np.float64)
    _check(lib().bc_brandes_plain(G.h, _p(S), S.size, _flags(ordered, engine_only), _p(out)))
    return out


def brandes_plain_dev(G: Graph, S_dev, out_dev, ordered: bool = False, engine_only: bool = False):
    """S_dev: int32 device tensor; out_dev: float64 device tensor of G.n entries."""
    _check(lib().bc_brandes_plain_dev(G.h, ctypes.c_void_p(S_dev.data_ptr()), S_dev.numel(),
                                      _flags(ordered, engine_only),
                                      ctypes.c_void_p(out_dev.data_ptr())))
    return out_dev


def brandes_plain_noalloc(G: Graph, S_dev, out_dev, ordered: bool = False):
    """bc_brandes_plain_noalloc: as brandes_plain_dev, with every buffer beyond S_dev and
    out_dev taken from the library's fixed device scratch array."""
    _check(lib().bc_brandes_plain_noalloc(G.h, ctypes.c_void_p(S_dev.data_ptr()), S_dev.numel(),
                                          BC_ORDERED if ordered else 0,
                                          ctypes.c_void_p(out_dev.data_ptr())))
    return out_dev


def noalloc_scratch_bytes() -> int:
    return int(lib().bc_noalloc_scratch_bytes())


def partition_lp(G: Graph, max_part: int = 0, rounds: int = 20, seed: int = 1406):
    """bc_partition_lp: (labels [n] int32, k) from size-constrained label propagation."""
    part = np.empty(G.n, np.int32)
    k = _i32(0)
    _check(lib().bc_partition_lp(G.h, int(max_part), int(rounds), ctypes.c_uint64(seed), _p(part),
                                 ctypes.byref(k)))
    return part, k.value


def brandes_pp_all(G: Graph, part, k: int, ordered: bool = False):
    """Brandes++All (bc_brandes_pp_all): all-pairs scores through k^2 skeletons."""
    part = _i32a(part)
    out = np.empty(G.n, np.float64)
    _check(lib().bc_brandes_pp_all(G.h, _p(part), int(k), BC_ORDERED if ordered else 0, _p(out)))
    return out


class Skeleton:
    """Skeleton handle (bc_partition_sk)."""

    def __init__(self, G: Graph, part, k: int, S):
        part = _i32a(part)
        S = _i32a(S)
        h = _P()
        _check(lib().bc_partition_sk(G.h, _p(part), int(k), _p(S), S.size, ctypes.byref(h)))
        self.h = h
        self.G = G

    def stats(self) -> dict:
        st = bc_sk_stats()
        _check(lib().bc_skeleton_stats(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in bc_sk_stats._fields_}

    def export(self) -> dict:
        st = self.stats()
        nsk = st["n_sk"]
        m = st["r_arcs"] + st["clique_arcs"]
        nodes = np.empty(nsk, np.int32)
        rp = np.empty(nsk + 1, np.int64)
        col = np.empty(max(m, 1), np.int32)
        ln = np.empty(max(m, 1), np.uint32)
        mu = np.empty(max(m, 1), np.uint64)
        nint = _i32(0)
        t = st["table_nnz"]
        tnode = np.empty(st["n"] + 1, np.int32)
        tptr = np.empty(st["n"] + 2, np.int64)
        tf = np.empty(max(t, 1), np.int32)
        td = np.empty(max(t, 1), np.uint32)
        ts = np.empty(max(t, 1), np.uint64)
        _check(lib().bc_skeleton_export(self.h, _p(nodes), _p(rp), _p(col), _p(ln), _p(mu),
                                        ctypes.byref(nint), _p(tnode), _p(tptr), _p(tf), _p(td),
                                        _p(ts)))
        ni = nint.value
        return {"nodes": nodes, "row_ptr": rp, "col": col[:m], "len": ln[:m], "mult": mu[:m],
                "tab_node": tnode[:ni], "tab_ptr": tptr[:ni + 1], "tab_f": tf[:t],
                "tab_d": td[:t], "tab_sigma": ts[:t]}

    def sssp_counts(self, src):
        src = _i32a(src)
        nsk = self.stats()["n_sk"]
        d = np.empty((src.size, nsk), np.int64)
        sig = np.empty((src.size, nsk), np.uint64)
        _check(lib().bc_skeleton_sssp_counts(self.h, _p(src), src.size, _p(d), _p(sig)))
        return d, sig

    def close(self):
        if self.h:
            lib().bc_skeleton_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def partition_sk(G: Graph, part, k: int, S) -> Skeleton:
    return Skeleton(G, part, k, S)


def brandes_pp(G: Graph, sk: Skeleton, ordered: bool = False, engine_only: bool = False):
    out = np.empty(G.n, np.float64)
    _check(lib().bc_brandes_pp(G.h, sk.h, _flags(ordered, engine_only), _p(out)))
    return out


def brandes_pp_dev(G: Graph, sk: Skeleton, out_dev, ordered: bool = False,
                   engine_only: bool = False):
    _check(lib().bc_brandes_pp_dev(G.h, sk.h, _flags(ordered, engine_only),
                                   ctypes.c_void_p(out_dev.data_ptr())))
    return out_dev


class Batch:
    """Many graphs in one device run (bc_batch_create / bc_batch_run)."""

    def __init__(self, graphs, stream=None):
        self.ns = [int(g.n) for g in graphs]
        structs, keep = [], []
        for g in graphs:
            s, k = _csr_struct(g)
            structs.append(s)
            keep.append(k)
        arr = (bc_csr * len(graphs))(*structs)
        parts = [_i32a(g.part) for g in graphs]
        Ss = [_i32a(g.S) for g in graphs]
        pp = (ctypes.c_void_p * len(graphs))(*[p.ctypes.data for p in parts])
        sp = (ctypes.c_void_p * len(graphs))(*[s.ctypes.data for s in Ss])
        ks = _i32a([g.k for g in graphs])
        nS = _i32a([s.size for s in Ss])
        h = _P()
        _check(lib().bc_batch_create(len(graphs), ctypes.cast(arr, _P), ctypes.cast(pp, _P),
                                     _p(ks), ctypes.cast(sp, _P), _p(nS), _stream(stream),
                                     ctypes.byref(h)))
        self.h = h

    def run(self, pp: bool = True, engine_only: bool = False, graph: bool = True, ordered: bool = False):
        """graph=False runs the pass eagerly instead of replaying its captured graph;
        ordered=True returns the ordered-pair sums (twice the default)."""
        outs = [np.empty(n, np.float64) for n in self.ns]
        ptrs = (ctypes.c_void_p * len(outs))(*[o.ctypes.data for o in outs])
        fl = ((BC_BATCH_PP if pp else BC_BATCH_PLAIN) | _flags(ordered, engine_only) |
              (0 if graph else BC_NO_GRAPH))
        _check(lib().bc_batch_run(self.h, fl, ctypes.cast(ptrs, _P)))
        return outs

    def close(self):
        if self.h:
            lib().bc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (bc_server_*, bc_query_*)."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 64):
        h = _P()
        _check(lib().bc_server_create(int(hbm_budget_bytes), int(max_inflight), ctypes.byref(h)))
        self.h = h
        self.ns = {}

    def add_graph(self, g) -> int:
        s, keep = _csr_struct(g)
        part = _i32a(g.part)
        gid = _i32(0)
        _check(lib().bc_server_add_graph(self.h, ctypes.byref(s), _p(part), int(g.k),
                                         ctypes.byref(gid)))
        self.ns[gid.value] = int(g.n)
        return gid.value

    def submit(self, gid: int, S, ordered: bool = False, engine_only: bool = False):
        """Returns a ticket, or None when the queue is full (BC_E_AGAIN)."""
        S = _i32a(S)
        t = _u64(0)
        rc = lib().bc_query_submit(self.h, int(gid), _p(S), S.size, _flags(ordered, engine_only),
                                   ctypes.byref(t))
        if rc == BC_E_AGAIN:
            return None
        _check(rc)
        return t.value

    def poll(self, ticket: int, n: int):
        out = np.empty(n, np.float64)
        done = _i32(0)
        _check(lib().bc_query_poll(self.h, _u64(ticket), _p(out), ctypes.byref(done)))
        return out if done.value else None

    def stats(self) -> dict:
        st = bc_server_stats()
        _check(lib().bc_server_stats_get(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in bc_server_stats._fields_}

    def close(self):
        if self.h:
            lib().bc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True):
    lib().bc_profile_enable(1 if on else 0)


def profile_reset():
    lib().bc_profile_reset()


def profile_read() -> dict:
    out = {}
    for k, name in enumerate(KERNELS):
        n = _i64(0)
        ms = ctypes.c_double(0)
        by = ctypes.c_double(0)
        _check(lib().bc_profile_read(k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        out[name] = {"launches": n.value, "ms": ms.value, "alg_bytes": by.value}
    return out


def exported_symbols():
    """Names declared in include/bcpp.h (used by the CPU-side export test)."""
    import re

    hdr = open(os.path.join(HERE, "..", "include", "bcpp.h")).read()
    pat = r"^(?:int|void|size_t|const char\*)\s+(bc_[a-z_]+)\s*\("
    return sorted(set(re.findall(pat, hdr, re.MULTILINE)))
