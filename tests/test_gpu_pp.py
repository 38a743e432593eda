"""GPU parity of Brandes++ (Build_SK, Dijkstra_SK, Brandes_SK, Centrality).

* The skeleton (frontiers, cut arcs, clique tuples, tables) equals the oracle's plain
  definition built from its Dijkstra_SK, exactly.
* Distances and path counts on the skeleton equal those of G between skeleton nodes,
  bit for bit (the claim after eq. multiparents).
* Brandes++ scores equal the oracle's plain target-set Brandes within 1e-9 relative,
  for any partition (partition invariance).
"""
import numpy as np
import pytest

import oracle
from paper_1406_4173_amd import inputs

from test_gpu_plain import PATHS, assert_scores

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bcpp():
    from paper_1406_4173_amd import bcpp as b

    b.lib()
    return b


def skeleton_matches_oracle(b, g, part, k, S):
    G = b.Graph(g)
    sk = b.partition_sk(G, part, k, S)
    ex = sk.export()
    ref = oracle.skeleton(g, part, k, S)
    nodes = ex["nodes"].astype(np.int64)
    assert sorted(nodes.tolist()) == ref["nodes"].tolist()
    arcs = {}
    rp = ex["row_ptr"]
    for f in range(nodes.size):
        for e in range(rp[f], rp[f + 1]):
            key = (int(nodes[f]), int(nodes[ex["col"][e]]))
            assert key not in arcs, "duplicate skeleton arc"
            arcs[key] = (int(ex["len"][e]), int(ex["mult"][e]))
    want = {k_: (w, 1) for k_, w in ref["R"].items()}
    want.update(ref["clique"])
    assert arcs == want
    tabs = {}
    tp = ex["tab_ptr"]
    for i, v in enumerate(ex["tab_node"]):
        row = {}
        for e in range(tp[i], tp[i + 1]):
            row[int(nodes[ex["tab_f"][e]])] = (int(ex["tab_d"][e]), int(ex["tab_sigma"][e]))
        if row:
            tabs[int(v)] = row
    assert tabs == ref["tables"]
    st = sk.stats()
    assert st["n_sk"] == nodes.size
    assert st["r_arcs"] == len(ref["R"]) and st["clique_arcs"] == len(ref["clique"])
    return G, sk


def test_skeleton_structure_small_graphs(bcpp):
    for seed in range(60):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 60))
        g = inputs.random_graph(3000 + seed, n, float(rng.choice([0.05, 0.1, 0.3])),
                                wmax=[None, 3, 7][seed % 3], k=int(rng.integers(1, 8)),
                                ns=int(rng.integers(0, max(1, n // 4))))
        skeleton_matches_oracle(bcpp, g, g.part, g.k, g.S)


def test_skeleton_structure_engine_dijkstra_sk(bcpp, monkeypatch):
    # the same skeletons with Dijkstra_SK on the multi-group engine instead of the
    # resident kernel
    monkeypatch.setenv("BCPP_RESIDENT", "0")
    for seed in range(20):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 60))
        g = inputs.random_graph(3000 + seed, n, float(rng.choice([0.05, 0.1, 0.3])),
                                wmax=[None, 3, 7][seed % 3], k=int(rng.integers(1, 8)),
                                ns=int(rng.integers(0, max(1, n // 4))))
        skeleton_matches_oracle(bcpp, g, g.part, g.k, g.S)


def test_skeleton_structure_planted(bcpp):
    g = inputs.planted_1k()
    S = inputs.random_targets(21, g.n, 40)
    skeleton_matches_oracle(bcpp, g, g.part, g.k, S)


def test_skeleton_preserves_distances_and_counts(bcpp):
    for seed, (n, p, wmax, k, ns) in enumerate([(80, 0.06, None, 5, 10), (120, 0.05, 4, 6, 12),
                                                 (300, 0.02, 3, 10, 30)]):
        g = inputs.random_graph(4000 + seed, n, p, wmax=wmax, k=k, ns=ns)
        G = bcpp.Graph(g)
        sk = bcpp.partition_sk(G, g.part, g.k, g.S)
        nodes = sk.export()["nodes"]
        src = [int(s) for s in g.S if s in set(nodes.tolist())]
        d, sig = sk.sssp_counts(src)
        for i, s in enumerate(src):
            od, osig = oracle.sssp(g, s)
            assert np.array_equal(d[i], od[nodes]), f"d_SK != d_G from {s}"
            assert np.array_equal(sig[i], osig[nodes]), f"sigma_SK != sigma_G from {s}"


@PATHS
def test_pp_small_random_graphs(bcpp, engine_only):
    for seed in range(150):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 50))
        g = inputs.random_graph(5000 + seed, n, float(rng.choice([0.04, 0.1, 0.25])),
                                wmax=[None, 3, 9][seed % 3], k=int(rng.integers(1, 9)))
        G = bcpp.Graph(g)
        sk = bcpp.partition_sk(G, g.part, g.k, g.S)
        want = oracle.bc(g, g.S)
        assert_scores(bcpp.brandes_pp(G, sk, engine_only=engine_only), want)
        assert_scores(bcpp.brandes_pp(G, sk, ordered=True, engine_only=engine_only), 2 * want)


@PATHS
def test_pp_partition_invariance(bcpp, engine_only):
    g = inputs.planted_1k()
    S = inputs.random_targets(31, g.n, 90)
    want = oracle.bc(g, S)
    G = bcpp.Graph(g)
    parts = {
        "planted": (g.part, g.k),
        "one part": (np.zeros(g.n, np.int32), 1),
        "singletons": (np.arange(g.n, dtype=np.int32), g.n),
        "random 37": (inputs.random_partition(1, g.n, 37), 37),
    }
    for name, (part, k) in parts.items():
        sk = bcpp.partition_sk(G, part, k, S)
        assert_scores(bcpp.brandes_pp(G, sk, engine_only=engine_only), want)


@PATHS
def test_pp_edge_cases(bcpp, engine_only):
    # isolated targets, a part with no frontier, a part made only of targets
    g = inputs.graph_from_edges(12, [0, 1, 2, 3, 5, 6, 8], [1, 2, 3, 4, 6, 7, 9])
    g.part = np.array([0, 0, 0, 1, 1, 2, 2, 2, 3, 3, 4, 5], np.int32)
    g.k = 6
    G = bcpp.Graph(g)
    for S in ([0, 4, 10, 11], [0, 4], [3, 4, 0], [10, 11], [], [2]):
        S = np.array(S, np.int32)
        sk = bcpp.partition_sk(G, g.part, g.k, S)
        assert_scores(bcpp.brandes_pp(G, sk, engine_only=engine_only), oracle.bc(g, S))
    with pytest.raises(bcpp.BcError):
        bcpp.partition_sk(G, g.part, 3, [0, 4])
    with pytest.raises(bcpp.BcError):
        bcpp.partition_sk(G, g.part, g.k, [0, 0])


@PATHS
def test_pp_overflow(bcpp, engine_only):
    g = inputs.grid(35, 35)
    G = bcpp.Graph(g)
    part = (np.arange(g.n) // 35 // 5).astype(np.int32)
    sk = bcpp.partition_sk(G, part, 7, [0, g.n - 1])
    with pytest.raises(bcpp.BcError) as ei:
        bcpp.brandes_pp(G, sk, engine_only=engine_only)
    assert ei.value.code == bcpp.BC_E_OVERFLOW


def test_identity_skeleton_equals_the_general_build(bcpp, monkeypatch):
    """Every node a target, in id order: G_SK is G less its isolated nodes (Sec. 5 with
    S = V), which the library then takes without building it. The skeleton it exports
    and the scores equal the general build's bit for bit: unit weights without isolated
    nodes (a grid in strips, G's own arrays), with one (planted_1k, arcs renumbered), and
    weighted (sbm_10k)."""
    grid = inputs.grid(30, 40)
    grid.part = (np.arange(grid.n) // 40 // 6).astype(np.int32)
    grid.k = 5
    grid.S = np.arange(grid.n, dtype=np.int32)
    planted = inputs.planted_1k()
    assert np.sum(np.diff(planted.row_ptr) == 0) >= 1
    for g in (grid, planted, inputs.sbm_10k()):
        assert np.array_equal(g.S, np.arange(g.n))
        got = {}
        for mode in ("1", "0"):
            monkeypatch.setenv("BCPP_SK_IDENTITY", mode)
            G = bcpp.Graph(g)
            sk = bcpp.partition_sk(G, g.part, g.k, g.S)
            got[mode] = (sk.export(), sk.stats(), bcpp.brandes_pp(G, sk))
        (ea, sa, ba), (eb, sb, bb) = got["1"], got["0"]
        for key in ea:
            assert np.array_equal(ea[key], eb[key]), key
        assert {k: v for k, v in sa.items() if k != "device_bytes"} == {
            k: v for k, v in sb.items() if k != "device_bytes"}
        assert np.array_equal(ba, bb)
    for seed in range(8):
        g = inputs.random_graph(77 + seed, 40, 0.06, wmax=[None, 3][seed % 2], k=4)
        g.S = np.arange(g.n, dtype=np.int32)
        skeleton_matches_oracle(bcpp, g, g.part, g.k, g.S)
    # every node isolated: an empty skeleton and zero scores
    g = inputs.empty(5)
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, np.zeros(5, np.int32), 1, np.arange(5))
    assert sk.stats()["n_sk"] == 0
    assert np.array_equal(bcpp.brandes_pp(G, sk), np.zeros(5))


def test_pp_near_overflow_grid_reports_none(bcpp):
    """34 x 35 grid, corner to corner: the largest path count is C(67, 33) < 2^64. With
    5-row strips as parts every interior row holds up to 70 table entries, so a row's
    entries span two rounds of the interior sweep, and products of counts over entries
    that are not tight may pass 2^64: none of that may be reported as overflow (eq.
    localcentrality sums only the tight entries), and the scores match the oracle."""
    g = inputs.grid(34, 35)
    G = bcpp.Graph(g)
    part = (np.arange(g.n) // 35 // 5).astype(np.int32)
    S = [0, g.n - 1]
    sk = bcpp.partition_sk(G, part, 7, S)
    assert max(len(r) for r in oracle.skeleton(g, part, 7, S)["tables"].values()) > 64
    assert_scores(bcpp.brandes_pp(G, sk), oracle.bc(g, S))


@PATHS
def test_pp_planted_1k_full(bcpp, engine_only):
    g = inputs.planted_1k()
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, g.S)
    assert_scores(bcpp.brandes_pp(G, sk, engine_only=engine_only), oracle.bc(g, g.S))


@PATHS
def test_pp_sbm_10k_full(bcpp, engine_only):
    g = inputs.sbm_10k()
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, g.S)
    assert_scores(bcpp.brandes_pp(G, sk, engine_only=engine_only), oracle.bc(g, g.S))


@PATHS
def test_pp_smallcut_100k(bcpp, engine_only):
    g = inputs.smallcut_100k()
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, g.S)
    want = oracle.bc(g, g.S)
    assert_scores(bcpp.brandes_pp(G, sk, engine_only=engine_only), want)
    assert_scores(bcpp.brandes_plain(G, g.S), want)


def test_pp_pareto_100k(bcpp):
    g = inputs.pareto_100k()
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, g.S)
    want = oracle.bc(g, g.S)
    assert_scores(bcpp.brandes_pp(G, sk), want)
    assert_scores(bcpp.brandes_plain(G, g.S), want)


def test_pp_bucket_and_scan_steps_agree(bcpp, monkeypatch):
    """Brandes++ on a skeleton too large for LDS (bucket frontiers in Brandes_SK): the
    dense-step threshold moves time only, never a bit of the result."""
    rng = inputs.rng_for(inputs.SEED_BASE + 92)
    g = inputs._community_graph(rng, 40000, 800, 8.0, 0.94, 4, "bucket40k")
    g.S = np.sort(rng.choice(g.n, 120, replace=False)).astype(np.int32)
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, g.S)
    assert sk.stats()["n_sk"] > 13000
    got = {}
    for shift in ("0", "63"):
        monkeypatch.setenv("BCPP_TUNE_DENSE_SHIFT", shift)
        got[shift] = bcpp.brandes_pp(G, sk)
    assert np.array_equal(got["0"], got["63"])
    assert_scores(got["0"], oracle.bc(g, g.S))


def test_dijkstra_sk_launch_shapes_change_no_bit(bcpp, monkeypatch):
    """Dijkstra_SK's launch shapes (thread classes, sources per group) are free choices:
    with every part's sources dealt 8 to a group and the widest workgroups, and with
    64 to a group on the narrowest, the skeleton equals the oracle's exactly and the
    Brandes++ scores are bitwise those of the tuned shapes."""
    g = inputs.planted_1k()
    S = inputs.random_targets(23, g.n, 40)
    G = bcpp.Graph(g)
    tuned = bcpp.brandes_pp(G, bcpp.partition_sk(G, g.part, g.k, S))
    for small, mid, work in (("0", "0", "1"), ("100000", "100000", "0")):
        monkeypatch.setenv("BCPP_TUNE_DSK_SMALL", small)
        monkeypatch.setenv("BCPP_TUNE_DSK_MID", mid)
        monkeypatch.setenv("BCPP_TUNE_DSK_WORK", work)
        G2, sk = skeleton_matches_oracle(bcpp, g, g.part, g.k, S)
        assert np.array_equal(bcpp.brandes_pp(G2, sk), tuned)
    assert_scores(tuned, oracle.bc(g, S))


@pytest.mark.parametrize("intra", [0.9, 0.998])
def test_pp_small_cut_sweep_graphs(bcpp, intra):
    # the two ends of the small-cut sweep (100,000 nodes, communities of 20): a large
    # skeleton with small tables, and a small skeleton with large tables
    g = inputs.p1_graph(intra)
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, g.S)
    want = oracle.bc(g, g.S)
    assert_scores(bcpp.brandes_pp(G, sk), want)
    assert_scores(bcpp.brandes_plain(G, g.S), want)


def test_pp_skeletons_alive_together_and_freed_out_of_order(bcpp):
    """Skeletons of three graphs of different sizes are built while others are alive
    and freed out of order (device memory freed by one is often handed to the next);
    every Brandes++ result equals that graph's first one bit for bit, and the first
    ones equal the oracle."""
    rng = inputs.rng_for(inputs.SEED_BASE + 95)
    graphs = [inputs.planted_1k()]
    for n, k in ((30000, 600), (8000, 160)):
        g = inputs._community_graph(rng, n, k, 8.0, 0.97, 4, "recycle")
        g.S = np.sort(rng.choice(n, 50, replace=False)).astype(np.int32)
        graphs.append(g)
    Gs = [bcpp.Graph(g) for g in graphs]
    first = {}
    alive = []
    for step, i in enumerate([1, 0, 2, 1, 2, 0, 2, 1, 0]):
        g = graphs[i]
        sk = bcpp.partition_sk(Gs[i], g.part, g.k, g.S)
        got = bcpp.brandes_pp(Gs[i], sk)
        if i in first:
            assert np.array_equal(got, first[i]), f"graph {i} at step {step}"
        else:
            assert_scores(got, oracle.bc(g, g.S))
            first[i] = got
        alive.append(sk)
        if step % 3 != 0:
            alive.pop(0).close()
        if step % 4 == 3:
            alive.pop().close()
    for sk in alive:
        sk.close()


def test_pp_lds_skeleton_with_wide_cliques(bcpp):
    """A skeleton held in LDS with the tight-arc bitmap, wide rows and path
    multiplicities: 2,000 nodes in 4 parts, degree 12, 10% of edges cut, weights 1..2,
    40 targets. Its 1,531 frontier nodes have about 50 arcs each (up to 153), and
    clique arcs carry up to 4 shortest paths."""
    rng = inputs.rng_for(inputs.SEED_BASE + 99, 2000, 4)
    g = inputs._community_graph(rng, 2000, 4, 12.0, 0.9, 2, "cliques")
    g.S = np.sort(rng.choice(g.n, 40, replace=False)).astype(np.int32)
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, g.S)
    st = sk.stats()
    assert st["n_sk"] == 1531 and st["r_arcs"] + st["clique_arcs"] >= 6 * st["n_sk"]
    assert_scores(bcpp.brandes_pp(G, sk), oracle.bc(g, g.S))


def test_pp_split_interior_rows(bcpp, monkeypatch):
    """Groups of 4 to 64 sources, or with at least 8192 table rows, sweep their interior
    rows (Sec. 5, eq. localcentrality) in a kernel of their own after the resident
    launch. Its scores equal the oracle's within 1e-9, and the in-kernel sweep's
    (BCPP_ISPLIT=0): parts of 250 and of 4,000 nodes, unit and integer weights, 6
    sources per group in 8 lanes, 4 per group, and one source per group over 38,000
    rows; a second run gives the same bits."""
    cases = []
    for seed, wmax in ((0, None), (1, 4)):
        g = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 99, seed), inputs.equal_sizes(3000, 12), 0.012, 600,
                       wmax, "split3k")
        cases.append((g, inputs.random_targets(70 + seed, g.n, 1500)))  # 6 sources per group
    g = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 99, 2), inputs.equal_sizes(12000, 3), 0.002, 3000, 3,
                   "split12k")
    cases.append((g, inputs.random_targets(72, g.n, 1024)))  # 4 sources per group
    g = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 99, 3), inputs.equal_sizes(40000, 2000), 0.3, 1500, 3,
                   "split40k")
    cases.append((g, inputs.random_targets(73, g.n, 60)))  # one source per group, many rows
    for g, S in cases:
        G = bcpp.Graph(g)
        sk = bcpp.partition_sk(G, g.part, g.k, S)
        assert sk.stats()["table_nnz"] > 0
        want = oracle.bc(g, S)
        monkeypatch.setenv("BCPP_ISPLIT", "1")
        a = bcpp.brandes_pp(G, sk)
        assert np.array_equal(a, bcpp.brandes_pp(G, sk))
        monkeypatch.setenv("BCPP_ISPLIT", "0")
        b = bcpp.brandes_pp(G, sk)
        assert_scores(a, want)
        assert_scores(b, want)
        assert_scores(a, b)


def test_pp_split_interior_64_sources_per_group(bcpp, monkeypatch):
    """64 sources per group (|S| = 16,384: rows of 64 threads, one per wave's lane): the
    split interior sweep against plain Brandes on the same targets (itself pinned to the
    oracle elsewhere; the oracle takes most of a minute here) and against the in-kernel
    sweep, within 1e-9."""
    # sparse blocks (mean degree about 2.5), so that many non-targets keep no target
    # neighbour and stay interior
    g = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 99, 4), inputs.equal_sizes(40000, 800), 0.05, 2000, None,
                   "split40k_sparse")
    S = inputs.random_targets(74, g.n, 16384)
    G = bcpp.Graph(g)
    sk = bcpp.partition_sk(G, g.part, g.k, S)
    assert sk.stats()["table_nnz"] > 0
    monkeypatch.setenv("BCPP_ISPLIT", "1")
    a = bcpp.brandes_pp(G, sk)
    monkeypatch.setenv("BCPP_ISPLIT", "0")
    b = bcpp.brandes_pp(G, sk)
    plain = bcpp.brandes_plain(G, S)
    assert_scores(a, plain)
    assert_scores(b, plain)
