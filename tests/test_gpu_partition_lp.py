"""GPU checks of the device partitioner (bc_partition_lp): label for label equal to
the numpy statement of its rule; a valid partition; Brandes++ over it matches the
oracle (the scores do not depend on the partition, Sec. 5)."""
import numpy as np
import pytest

import oracle
from lp_reference import label_propagation
from paper_1406_4173_amd import inputs

from test_gpu_plain import assert_scores

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bcpp():
    from paper_1406_4173_amd import bcpp as b

    b.lib()
    return b


CASES = [("planted_1k", 0, 20, 1), ("planted_1k", 150, 20, 2), ("sbm_10k", 300, 24, 3), ("isolated", 8, 12, 4)]


@pytest.mark.parametrize("name,cap,rounds,seed", CASES, ids=[f"{c[0]}-cap{c[1]}" for c in CASES])
def test_partition_lp_equals_reference(bcpp, name, cap, rounds, seed):
    if name == "isolated":
        g = inputs.random_graph(9300, 300, 0.006, wmax=3)
    else:
        g = inputs.CONFIGS[name]()
    part, k = bcpp.partition_lp(bcpp.Graph(g), cap, rounds, seed)
    want, wk = label_propagation(g, cap, rounds, seed)
    assert k == wk
    assert np.array_equal(part, want)
    assert part.min() == 0 and part.max() == k - 1 and np.unique(part).size == k


def test_brandes_pp_over_the_device_partition(bcpp):
    """Brandes++ over the partitioner's output matches the oracle. On sbm_10k (degree 10,
    90% of edges inside its 40 planted communities) the partition cuts at most 1.5x the
    planted share of edges; on planted_1k (degree 6.6, sparse communities) label
    propagation leaves many small parts, which only costs speed."""
    for g, S, cap, bound in ((inputs.planted_1k(), inputs.random_targets(41, 1000, 60), 200, None),
                             (inputs.sbm_10k(), inputs.random_targets(42, 10000, 40), 400, 1.5)):
        G = bcpp.Graph(g)
        part, k = bcpp.partition_lp(G, cap, 48, 5)
        sk = bcpp.partition_sk(G, part, k, S)
        assert_scores(bcpp.brandes_pp(G, sk), oracle.bc(g, S))
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        cut = np.mean(part[src] != part[g.col])
        planted = np.mean(g.part[src] != g.part[g.col])
        if bound:
            assert cut < bound * planted, (cut, planted)
