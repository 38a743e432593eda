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
