"""GPU parity of the batched form: many graphs in one device run.

Each graph's scores must match the oracle within 1e-9, and must equal (bit for bit) the
scores of the same graph run alone: the graph gets the same groups of sources in the
same order either way.
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


def mixed_graphs():
    out = []
    for seed in range(10):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 70))
        out.append(inputs.random_graph(7000 + seed, n, float(rng.choice([0.05, 0.1, 0.2])),
                                       wmax=[None, 4][seed % 2], k=int(rng.integers(1, 6))))
    out.append(inputs.empty(5))
    out[-1].part = np.zeros(5, np.int32)
    out[-1].k = 1
    out[-1].S = np.array([1, 3], np.int32)
    return out


@PATHS
@pytest.mark.parametrize("pp", [False, True])
def test_batch_mixed_graphs(bcpp, pp, engine_only):
    gs = mixed_graphs()
    B = bcpp.Batch(gs)
    res = B.run(pp=pp, engine_only=engine_only)
    for g, got in zip(gs, res):
        assert_scores(got, oracle.bc(g, g.S))


@PATHS
@pytest.mark.parametrize("pp", [False, True])
def test_batch_item_equals_alone(bcpp, pp, engine_only):
    gs = inputs.batch_256(12)
    res = bcpp.Batch(gs).run(pp=pp, engine_only=engine_only)
    for g, got in zip(gs, res):
        G = bcpp.Graph(g)
        if pp:
            alone = bcpp.brandes_pp(G, bcpp.partition_sk(G, g.part, g.k, g.S), engine_only=engine_only)
        else:
            alone = bcpp.brandes_plain(G, g.S, engine_only=engine_only)
        assert np.array_equal(got, alone)


@pytest.mark.parametrize("pp", [False, True])
def test_batch_resident_and_engine_graphs_together(bcpp, pp):
    # a graph too large for LDS (engine) between graphs that fit (resident kernel)
    # (20,000 nodes with 15,000 cut edges: its skeleton too has more nodes than LDS holds)
    big = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 96, 0), inputs.equal_sizes(20000, 40),
                     4.0 / 499, 15000, 3, "big20k")
    big.S = inputs.random_targets(33, big.n, 25)
    gs = mixed_graphs()[:4] + [big] + mixed_graphs()[4:]
    res = bcpp.Batch(gs).run(pp=pp)
    for g, got in zip(gs, res):
        assert_scores(got, oracle.bc(g, g.S))


def test_batch_256_full(bcpp):
    gs = inputs.batch_256()
    B = bcpp.Batch(gs)
    for pp in (True, False):
        res = B.run(pp=pp)
        for g, got in zip(gs, res):
            assert_scores(got, oracle.bc(g, g.S))


def test_batch_plain_graph_replays_match_eager(bcpp):
    # plain Brandes over a batch replays one captured HIP graph; every replay must equal
    # the eager run bit for bit, with other eager work and synchronisations in between
    gs = inputs.batch_256(24)
    B = bcpp.Batch(gs)
    eager = B.run(pp=False, graph=False)
    for g, got in zip(gs, eager):
        assert_scores(got, oracle.bc(g, g.S))
    other = inputs.planted_1k()
    Go = bcpp.Graph(other)
    for rep in range(4):
        res = B.run(pp=False)
        for a, b in zip(res, eager):
            assert np.array_equal(a, b), f"replay {rep} differs from the eager run"
        bcpp.brandes_plain(Go, other.S[: 40 + rep])
        bcpp.Batch(gs[:3]).run(pp=True)


def test_batch_pp_graph_replays_match_eager(bcpp):
    # Brandes++ over a batch replays one captured HIP graph holding the whole pipeline
    # (Build_SK, Dijkstra_SK, assembly, Brandes_SK + Centrality, reduction); every
    # replay must equal the eager run bit for bit, with eager runs of the same batch
    # (which use the union graph's own workspaces) and other work in between
    big = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 96, 0), inputs.equal_sizes(20000, 40),
                     4.0 / 499, 15000, 3, "big20k")
    big.S = inputs.random_targets(33, big.n, 25)
    gs = inputs.batch_256(20) + [big] + mixed_graphs()
    B = bcpp.Batch(gs)
    eager = B.run(pp=True, graph=False)
    for g, got in zip(gs, eager):
        assert_scores(got, oracle.bc(g, g.S))
    other = inputs.planted_1k()
    Go = bcpp.Graph(other)
    for rep in range(4):
        res = B.run(pp=True)
        for a, b in zip(res, eager):
            assert np.array_equal(a, b), f"replay {rep} differs from the eager run"
        again = B.run(pp=True, graph=False)
        for a, b in zip(again, eager):
            assert np.array_equal(a, b)
        bcpp.brandes_pp(Go, bcpp.partition_sk(Go, other.part, other.k, other.S[: 40 + rep]))
        B.run(pp=False)


@pytest.mark.parametrize("graph", [True, False], ids=["replay", "eager"])
def test_batch_ordered_is_twice_unordered(bcpp, graph):
    # BC_ORDERED gives the ordered-pair sums, exactly twice the unordered scores, for
    # both passes (scaling by 2 is exact in fp64)
    gs = inputs.batch_256(10)
    B = bcpp.Batch(gs)
    for pp in (False, True):
        a = B.run(pp=pp, graph=graph)
        b = B.run(pp=pp, graph=graph, ordered=True)
        for x, y, g in zip(a, b, gs):
            assert np.array_equal(y, 2.0 * x)
            assert_scores(y, oracle.bc(g, g.S, True))


def test_batch_pp_split_interior_replays(bcpp):
    """Graphs whose Brandes_SK groups sweep their interior rows in the kernels of their
    own (groups of 6 sources in 8 lanes; one source over 37,000 rows) inside a batch:
    the captured pass replays bit for bit equal to its eager run, each graph equals its
    run alone, and the scores equal the oracle's within 1e-9."""
    wide = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 99, 0), inputs.equal_sizes(3000, 12), 0.012, 600,
                      None, "split3k")
    wide.S = inputs.random_targets(70, wide.n, 1500)
    narrow = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 99, 3), inputs.equal_sizes(40000, 2000), 0.3, 1500, 3,
                        "split40k")
    narrow.S = inputs.random_targets(73, narrow.n, 60)
    gs = [wide] + inputs.batch_256(6) + [narrow]
    B = bcpp.Batch(gs)
    eager = B.run(pp=True, graph=False)
    for g, got in zip(gs, eager):
        assert_scores(got, oracle.bc(g, g.S))
        G = bcpp.Graph(g)
        assert np.array_equal(got, bcpp.brandes_pp(G, bcpp.partition_sk(G, g.part, g.k, g.S)))
    for rep in range(3):
        res = B.run(pp=True)
        for a, b in zip(res, eager):
            assert np.array_equal(a, b), f"replay {rep} differs from the eager run"
