"""GPU parity of Brandes++All (Sec. 6, Alg. 3): the k^2 skeleton passes sum to the
all-pairs scores (S = V) of the oracle within 1e-9, for any partition."""
import numpy as np
import pytest

import oracle
from paper_1406_4173_amd import inputs

from test_gpu_plain import assert_scores

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bcpp():
    from paper_1406_4173_amd import bcpp as b

    b.lib()
    return b


def test_pp_all_small_random_graphs(bcpp):
    for seed in range(40):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 40))
        g = inputs.random_graph(9100 + seed, n, float(rng.choice([0.05, 0.12, 0.3])),
                                wmax=[None, 3, 8][seed % 3], k=int(rng.integers(1, 7)))
        G = bcpp.Graph(g)
        V = np.arange(g.n, dtype=np.int32)
        want = oracle.bc(g, V)
        assert_scores(bcpp.brandes_pp_all(G, g.part, g.k), want)
        if seed % 4 == 0:
            assert_scores(bcpp.brandes_pp_all(G, g.part, g.k, ordered=True), 2 * want)


def test_pp_all_partitions_planted_1k(bcpp):
    g = inputs.planted_1k()
    G = bcpp.Graph(g)
    want = oracle.bc(g, np.arange(g.n, dtype=np.int32))
    assert_scores(bcpp.brandes_pp_all(G, g.part, g.k), want)
    assert_scores(bcpp.brandes_pp_all(G, np.zeros(g.n, np.int32), 1), want)
    assert_scores(bcpp.brandes_pp_all(G, inputs.random_partition(3, g.n, 5), 5), want)


def test_pp_all_singletons_and_unused_labels(bcpp):
    g = inputs.random_graph(9200, 24, 0.15, wmax=4)
    G = bcpp.Graph(g)
    want = oracle.bc(g, np.arange(g.n, dtype=np.int32))
    assert_scores(bcpp.brandes_pp_all(G, np.arange(g.n, dtype=np.int32), g.n), want)
    part = (np.arange(g.n) % 3 * 2).astype(np.int32)  # labels 0, 2, 4 of k = 6
    assert_scores(bcpp.brandes_pp_all(G, part, 6), want)
    with pytest.raises(bcpp.BcError):
        bcpp.brandes_pp_all(G, part, 4)


def test_pp_all_shared_build_equals_per_pass_builds(bcpp, monkeypatch):
    """Build_SK once (Alg. 3): the passes that take the shared Dijkstra_SK results of
    the parts other than P_i and P_j, and run their Brandes_SK groups together, give the
    scores of k^2 independent builds and launches bit for bit, also when the passes are
    split over several launches (a pending-state cap of 0 MB: one launch per pass)."""
    g2 = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 97, 0), inputs.equal_sizes(3000, 6),
                    0.01, 900, 4, "sbm3k")
    g3 = inputs.random_graph(9300, 60, 0.08, wmax=5, k=4)
    for g in (inputs.planted_1k(), g2, g3):
        G = bcpp.Graph(g)
        got = []
        for reuse, cap in (("0", None), ("1", None), ("1", "0")):
            monkeypatch.setenv("BCPP_PPALL_REUSE", reuse)
            if cap is None:
                monkeypatch.delenv("BCPP_PPALL_PENDING_MB", raising=False)
            else:
                monkeypatch.setenv("BCPP_PPALL_PENDING_MB", cap)
            got.append(bcpp.brandes_pp_all(G, g.part, g.k))
        assert np.array_equal(got[0], got[1])
        assert np.array_equal(got[0], got[2])
        if g.n <= 1000:
            assert_scores(got[1], oracle.bc(g, np.arange(g.n, dtype=np.int32)))
