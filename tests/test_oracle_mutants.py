"""Planted mistakes in the oracle must fail its pins.

Each case copies oracle/oracle_bc.c to a temporary directory, applies one plausible
mistake (a dropped term, a wrong index, a transposed operand, a lost check), builds
the copy with gcc and runs the pin checks against it. The committed oracle is never
modified; the mutants run on the CPU only.
"""
import os
from math import comb

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_1406_4173_amd import inputs

MUTANTS = {
    "drop_indicator": ("((double)in_s[v] + delta[v])", "(delta[v])"),
    "indicator_always_one": ("((double)in_s[v] + delta[v])", "(1.0 + delta[v])"),
    "no_halving": ("C_out[v] *= 0.5;", "C_out[v] *= 1.0;"),
    "source_accumulated": ("if (u != s) C_out[u] += delta[u];", "C_out[u] += delta[u];"),
    "ratio_transposed": ("(double)sigma[u] / (double)sigma[v]",
                         "(double)sigma[v] / (double)sigma[u]"),
    "bfs_sigma_assign": ("uint64_t t = sigma[v] + sigma[u];\n                    if (t < sigma[v]) return ORACLE_OVERFLOW;\n                    sigma[v] = t;\n                }\n            }\n        }\n    } else",
                         "uint64_t t = sigma[u];\n                    sigma[v] = t;\n                }\n            }\n        }\n    } else"),
    "dijkstra_no_reset": ("sigma[v] = parent_ok ? sigma[u] : 0;",
                          "sigma[v] += parent_ok ? sigma[u] : 0;"),
    "backward_not_tight": ("d[v] == d[u] + len", "d[v] > d[u]"),
    "frontier_parents_allowed": ("frontier[u] == 0 || u == s", "1"),
    "source_parent_excluded": ("frontier[u] == 0 || u == s", "frontier[u] == 0"),
    "no_overflow_check": ("if (t < sigma[v]) return ORACLE_OVERFLOW;", "(void)0;"),
    "weight_ignored": ("int64_t nd = d[u] + (int64_t)w[e];", "int64_t nd = d[u] + 1;"),
    "part_boundary_ignored": ("if (label != NULL && label[v] != label[s]) continue;", ""),
}


def _pins(L):
    """The oracle pins, in a compact form; raises on the first failure."""
    for seed in range(300):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 11))
        g = inputs.random_graph(seed, n, float(rng.choice([0.3, 0.5])),
                                wmax=[None, 3][seed % 2])
        exact = bf.to_float(bf.bc_bruteforce(g, g.S))
        got = oracle.bc(g, g.S, L=L)
        assert np.allclose(got, exact, rtol=1e-12, atol=1e-12)
    g = inputs.star(7)
    assert oracle.bc(g, np.arange(7), L=L)[0] == 15
    g = inputs.grid(5, 6)
    _, sig = oracle.sssp(g, 0, L=L)
    assert int(sig[-1]) == comb(9, 4)
    g = inputs.grid(35, 35)
    try:
        oracle.sssp(g, 0, L=L)
        raise AssertionError("overflow not detected")
    except oracle.OracleError as e:
        assert e.code == oracle.OVERFLOW
    for seed in range(60):
        rng = np.random.default_rng(1000 + seed)
        n = int(rng.integers(3, 9))
        g = inputs.random_graph(500 + seed, n, 0.5, wmax=[None, 3][seed % 2],
                                k=int(rng.integers(1, 4)))
        lab = oracle.prime_labels(g.n, g.part, g.k, g.S[:1])
        fr = oracle.frontier_flags(g, lab)
        for f in np.nonzero(fr)[0]:
            d, sig = oracle.dijkstra_sk(g, lab, fr, int(f), L=L)
            ref = bf.restricted_counts(g, lab, fr, int(f))
            for v in range(g.n):
                if lab[v] != lab[f]:
                    assert d[v] == -1 and sig[v] == 0
                    continue
                dv, cv = ref[v]
                assert (d[v] == -1 and dv is None) or (d[v] == dv and int(sig[v]) == cv)


def test_unmutated_oracle_passes_pins(oracle_lib):
    _pins(oracle_lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    before, after = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert before in src, f"mutation site for {name} not found"
    mutated = src.replace(before, after)
    path = os.path.join(tmp_path, "mut.c")
    with open(path, "w") as f:
        f.write(mutated)
    so = oracle.build(out=os.path.join(tmp_path, "libmut.so"), src=path)
    L = oracle.lib(so)
    with pytest.raises((AssertionError, oracle.OracleError)):
        _pins(L)
