"""Bit-exact distances and path counts of the kernel that produces every score.

bc_sssp_counts and bc_skeleton_sssp_counts run the groups of a plain Brandes pass (or
of a Brandes_SK + Centrality pass on the skeleton) over the given sources, with the
full forward and backward sweeps, and export each source's d and sigma right after its
forward sweep (Sec. 3 eq. parentsall; Sec. 5 eq. multiparents). Every case below
compares them bit for bit with the oracle's counts on G: with the state in LDS (the
256-, 512- and 1024-thread classes), in device memory (bucket and scan steps), on
skeletons with multiplicities, and at the uint64 overflow boundary. The multi-group
engine (BCPP_RESIDENT=0) is checked on the same small cases.
"""
import numpy as np
import pytest

import oracle
from paper_1406_4173_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bcpp():
    from paper_1406_4173_amd import bcpp as b

    b.lib()
    return b


def check_graph_counts(b, g, src, G=None):
    G = G or b.Graph(g)
    d, sig = b.sssp_counts(G, src)
    assert d.shape == (len(src), g.n)
    for i, s in enumerate(src):
        od, osig = oracle.sssp(g, int(s))
        assert np.array_equal(d[i], od), f"distances differ from source {s}"
        assert np.array_equal(sig[i], osig), f"path counts differ from source {s}"
    return d, sig


def check_skeleton_counts(b, g, S, nsrc, G=None):
    """Skeleton counts (eq. multiparents, multiplicities of the clique arcs) from up to
    nsrc targets equal G's counts at the skeleton nodes."""
    G = G or b.Graph(g)
    sk = b.partition_sk(G, g.part, g.k, S)
    nodes = sk.export()["nodes"]
    on_sk = set(nodes.tolist())
    src = [int(s) for s in S if int(s) in on_sk][:nsrc]
    assert src
    d, sig = sk.sssp_counts(src)
    for i, s in enumerate(src):
        od, osig = oracle.sssp(g, s)
        assert np.array_equal(d[i], od[nodes]), f"d_SK != d_G from {s}"
        assert np.array_equal(sig[i], osig[nodes]), f"sigma_SK != sigma_G from {s}"
    return sk


@pytest.mark.parametrize("engine", [False, True], ids=["resident", "engine"])
def test_counts_small_graphs_both_back_ends(bcpp, monkeypatch, engine):
    if engine:
        monkeypatch.setenv("BCPP_RESIDENT", "0")
    for seed in range(30):
        g = inputs.random_graph(seed, 5 + seed % 20, 0.3, wmax=[None, 4][seed % 2])
        check_graph_counts(bcpp, g, np.arange(g.n))
    g = inputs.grid(9, 13)
    for ns in (1, 63, 64, 65, 117):
        check_graph_counts(bcpp, g, np.arange(ns) % g.n)


@pytest.mark.parametrize("n,deg", [(1500, 8.0), (4000, 8.0), (11000, 9.0)],
                         ids=["lds256", "lds512", "lds1024"])
def test_counts_lds_state_classes(bcpp, n, deg):
    """Ranges of each LDS thread class, weights 1..7, with the tight-arc bitmap."""
    rng = inputs.rng_for(inputs.SEED_BASE + 131, n)
    g = inputs._community_graph(rng, n, max(4, n // 100), deg, 0.9, 7, "lds")
    check_graph_counts(bcpp, g, np.sort(rng.choice(n, 40, replace=False)))


def test_counts_planted_1k_and_sbm_10k(bcpp):
    g = inputs.planted_1k()
    check_graph_counts(bcpp, g, inputs.random_targets(11, g.n, 130))
    g = inputs.sbm_10k()
    check_graph_counts(bcpp, g, inputs.random_targets(12, g.n, 300))


def test_counts_pareto_100k_device_memory_state(bcpp):
    """100,000 nodes: the one-source state lives in device memory (L2 atomics, bucket
    frontiers, the tight-arc bitmap in device memory)."""
    g = inputs.pareto_100k()
    check_graph_counts(bcpp, g, g.S[:24])


@pytest.mark.parametrize("shift", ["0", "63"])
def test_counts_device_memory_bucket_and_scan_steps(bcpp, monkeypatch, shift):
    """A 20,000-node range in device memory: dense-step threshold 0 (every step reads its
    bucket) and 63 (every step scans the range) give the oracle's counts bit for bit."""
    monkeypatch.setenv("BCPP_TUNE_DENSE_SHIFT", shift)
    rng = inputs.rng_for(inputs.SEED_BASE + 91, 4, 20000)
    g = inputs._community_graph(rng, 20000, 400, 8.0, 0.99, 4, "bucket")
    check_graph_counts(bcpp, g, np.sort(rng.choice(g.n, 20, replace=False)))


def test_counts_overflow_boundary(bcpp):
    """Grid path counts C(i+j, i): 34 x 35 fits in uint64, 35 x 35 must fail."""
    g = inputs.grid(34, 35)
    d, sig = check_graph_counts(bcpp, g, [0, g.n - 1, 17])
    assert int(sig[0][-1]) == 14226520737620288370  # C(67, 33)
    g = inputs.grid(35, 35)
    with pytest.raises(bcpp.BcError) as ei:
        bcpp.sssp_counts(bcpp.Graph(g), [0])
    assert ei.value.code == bcpp.BC_E_OVERFLOW


def test_skeleton_counts_lds_with_multiplicities(bcpp):
    """A skeleton held in LDS whose clique arcs carry several shortest paths each."""
    rng = inputs.rng_for(inputs.SEED_BASE + 99, 2000, 4)
    g = inputs._community_graph(rng, 2000, 4, 12.0, 0.9, 2, "cliques")
    S = np.sort(rng.choice(g.n, 40, replace=False)).astype(np.int32)
    sk = check_skeleton_counts(bcpp, g, S, 40)
    assert sk.export()["mult"].max() > 1
    g = inputs.planted_1k()
    check_skeleton_counts(bcpp, g, inputs.random_targets(21, g.n, 40), 40)


def test_skeleton_counts_pareto_100k_device_memory(bcpp):
    """pareto_100k's skeleton (about 74,000 nodes, state in device memory, multiplicities
    and tables) from 16 of its targets."""
    g = inputs.pareto_100k()
    sk = check_skeleton_counts(bcpp, g, g.S, 16)
    assert sk.stats()["n_sk"] > 13000 and sk.export()["mult"].max() > 1


def test_skeleton_counts_engine(bcpp, monkeypatch):
    monkeypatch.setenv("BCPP_RESIDENT", "0")
    for seed, (n, p, wmax, k, ns) in enumerate([(80, 0.06, None, 5, 10), (300, 0.02, 3, 10, 30)]):
        g = inputs.random_graph(4000 + seed, n, p, wmax=wmax, k=k, ns=ns)
        check_skeleton_counts(bcpp, g, g.S, ns)


@pytest.mark.parametrize("byte", ["1", "0"], ids=["byte-state", "device-state"])
def test_counts_large_ranges_both_state_layouts(bcpp, monkeypatch, byte):
    """Ranges beyond LDS keep their distance state as one byte per node in LDS when arcs
    are at most 63 long (else, or with BCPP_BYTE=0, in device memory): both layouts give
    the oracle's counts bit for bit, on G (weights 1..12 and 1..60) and on a skeleton."""
    monkeypatch.setenv("BCPP_BYTE", byte)
    for wmax, seed in ((12, 1), (60, 2)):
        rng = inputs.rng_for(inputs.SEED_BASE + 133, seed)
        g = inputs._community_graph(rng, 16000, 300, 7.0, 0.95, wmax, "layouts")
        S = np.sort(rng.choice(g.n, 12, replace=False)).astype(np.int32)
        check_graph_counts(bcpp, g, S)
    rng = inputs.rng_for(inputs.SEED_BASE + 134)
    g = inputs._community_graph(rng, 40000, 800, 8.0, 0.94, 4, "layouts_sk")
    S = np.sort(rng.choice(g.n, 60, replace=False)).astype(np.int32)
    sk = check_skeleton_counts(bcpp, g, S, 10)
    assert sk.stats()["n_sk"] > 13000
