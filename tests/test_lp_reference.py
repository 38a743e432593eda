"""CPU checks of the label-propagation reference rule (tests/lp_reference.py)."""
import numpy as np

from lp_reference import label_propagation, splitmix64
from paper_1406_4173_amd import inputs


def test_splitmix64_first_output():
    # the generator seeded with 0 yields this first (a commonly quoted value)
    assert int(splitmix64(0)) == 0xE220A8397B1DCDAF


def test_disjoint_cliques_become_one_part_each():
    # 6 disjoint 5-cliques: once any node of a clique moves, its clique-mates follow;
    # after enough rounds every clique holds one label and no label spans two cliques
    u, v = [], []
    for c in range(6):
        for a in range(5):
            for b in range(a + 1, 5):
                u.append(5 * c + a)
                v.append(5 * c + b)
    g = inputs.graph_from_edges(30, u, v)
    part, k = label_propagation(g, 0, 40, 7)
    assert k == 6
    for c in range(6):
        assert len(set(part[5 * c:5 * c + 5].tolist())) == 1


def test_size_cap_and_determinism():
    g = inputs.planted_1k()
    p1, k1 = label_propagation(g, 100, 20, 3)
    p2, k2 = label_propagation(g, 100, 20, 3)
    assert k1 == k2 and np.array_equal(p1, p2)
    assert p1.min() == 0 and p1.max() == k1 - 1 and np.unique(p1).size == k1
    p3, _ = label_propagation(g, 0, 20, 4)
    assert not np.array_equal(p1, p3)
