"""The skeleton structure that the paper's Figure 1 caption spells out (Sec. 4)."""
import json
import os

import numpy as np

import oracle
from paper_1406_4173_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    fx = json.load(open(os.path.join(HERE, "golden", "figure1_skeleton.json")))
    names = fx["names"]
    idx = {s: i for i, s in enumerate(names)}
    u = [idx[a] for a, _ in fx["edges"]]
    v = [idx[b] for _, b in fx["edges"]]
    g = inputs.graph_from_edges(len(names), u, v)
    part = np.array([fx["parts"][s] for s in names], np.int32)
    return fx, idx, g, part


def test_figure1_skeleton_structure(oracle_lib):
    fx, idx, g, part = load()
    sk = oracle.skeleton(g, part, int(part.max()) + 1, np.array([], np.int32), L=oracle_lib)
    fr = {int(v) for v in sk["nodes"]}
    assert fr == {idx[s] for s in fx["expect_frontier_of_part0"] + fx["expect_frontier_other"]}
    R = {tuple(sorted(e)) for e in sk["R"]}
    assert R == {tuple(sorted((idx[a], idx[b]))) for a, b in fx["expect_R_undirected"]}
    clique0 = {tuple(sorted(e)) for e in sk["clique"] if part[e[0]] == 0}
    assert clique0 == {tuple(sorted((idx[a], idx[b]))) for a, b in fx["expect_clique_part0"]}
    # the clique tuples are symmetric (<d, sigma> does not depend on the direction)
    for (f, q), t in sk["clique"].items():
        assert sk["clique"][(q, f)] == t
