"""The seeded input generators (CPU): every workload has the documented shape (sizes,
part structure, degree, share of edges inside a community, weight range, target set)
and is a valid symmetric CSR (sorted rows, no self-loops or duplicates, each weight
stored in both arcs). The generators hold no method arithmetic; these checks pin the
recipe that the parity tests and the bench depend on."""
import numpy as np
import pytest

from paper_1406_4173_amd import inputs


def check_csr(g):
    rp = np.asarray(g.row_ptr, np.int64)
    col = np.asarray(g.col, np.int64)
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp))
    assert np.all((col >= 0) & (col < g.n)) and np.all(u != col)
    key = u * g.n + col
    assert np.all(np.diff(key) > 0), "rows unsorted or duplicate arcs"
    rev = col * g.n + u
    order = np.argsort(rev, kind="stable")
    assert np.array_equal(rev[order], key), "asymmetric CSR"
    if g.w is not None:
        w = np.asarray(g.w)
        assert np.all(w >= 1)
        assert np.array_equal(w[order], w), "arc and reverse arc differ in weight"


def intra_share(g):
    u, v, _ = g.edges()
    return float(np.mean(g.part[u] == g.part[v]))


def check_targets(g, count):
    S = np.asarray(g.S)
    assert S.size == count and np.unique(S).size == count
    assert S.min() >= 0 and S.max() < g.n


def part_sizes(g):
    return np.bincount(np.asarray(g.part), minlength=g.k)


def test_planted_1k():
    g = inputs.planted_1k()
    check_csr(g)
    assert (g.n, g.m, g.k) == (1000, 3309, 8) and g.w is None
    assert np.all(part_sizes(g) == 125)
    assert np.array_equal(np.asarray(g.S), np.arange(1000))


def test_sbm_10k():
    g = inputs.sbm_10k()
    check_csr(g)
    assert (g.n, g.m, g.k) == (10000, 50025, 40)
    assert np.all(part_sizes(g) == 250)
    assert g.w.min() == 1 and g.w.max() == 10
    assert abs(2 * g.m / g.n - 10) < 0.3 and abs(intra_share(g) - 0.9) < 0.01
    assert np.array_equal(np.asarray(g.S), np.arange(10000))


def test_pareto_100k():
    g = inputs.pareto_100k()
    check_csr(g)
    assert (g.n, g.m, g.k) == (100000, 400264, 500)
    sizes = part_sizes(g)
    assert sizes.sum() == 100000 and sizes.min() >= 2 and sizes.max() > 10 * np.median(sizes)
    assert g.w.min() == 1 and g.w.max() == 4
    assert abs(2 * g.m / g.n - 8) < 0.2 and abs(intra_share(g) - 0.85) < 0.01
    check_targets(g, 2000)


def test_smallcut_100k():
    g = inputs.smallcut_100k()
    check_csr(g)
    assert (g.n, g.k) == (100000, 2000) and np.all(part_sizes(g) == 50)
    assert g.w.min() == 1 and g.w.max() == 4
    assert abs(2 * g.m / g.n - 8) < 0.2 and abs(intra_share(g) - 0.99) < 0.002
    check_targets(g, 200)


@pytest.mark.parametrize("intra", inputs.P1_INTRA)
def test_small_cut_sweep_graph(intra):
    g = inputs.p1_graph(intra)
    check_csr(g)
    assert (g.n, g.k) == (100000, 5000) and np.all(part_sizes(g) == 20)
    assert abs(2 * g.m / g.n - 8) < 0.2 and abs(intra_share(g) - intra) < 0.003
    check_targets(g, 200)


def test_batch_256():
    gs = inputs.batch_256()
    assert len(gs) == 256
    assert sum(g.n for g in gs) == 366612 and sum(len(g.S) for g in gs) == 43731
    for g in gs:
        check_csr(g)
        assert 200 <= g.n <= 5000 and 4 <= g.k <= 32 and g.w is None
        sizes = part_sizes(g)
        assert sizes.max() - sizes.min() <= 1
        assert 5.0 <= 2 * g.m / g.n <= 13.0
        ns = len(g.S)
        assert np.unique(g.S).size == ns and max(2, int(0.05 * g.n) - 1) <= ns <= int(0.20 * g.n) + 1
    share = np.mean([intra_share(g) for g in gs])
    assert abs(share - 0.9) < 0.01


def test_serving_pool_and_stream():
    pool = inputs.serving_pool()
    assert len(pool) == 64
    for gi, g in enumerate(pool):
        check_csr(g)
        assert 1000 <= g.n <= 50000 and g.k == max(4, int(round(g.n / 200)))
        assert (g.w is None) == (gi % 2 == 0)
        if g.w is not None:
            assert g.w.min() >= 1 and g.w.max() <= 10
    stream = inputs.serving_stream([g.n for g in pool], rate=200.0, seconds=5.0)
    t = np.array([a for a, _, _ in stream])
    assert np.all(np.diff(t) > 0) and t[-1] < 5.0
    assert 800 <= len(stream) <= 1200  # Poisson(1000)
    for _, gi, S in stream:
        n = pool[gi].n
        assert np.unique(S).size == S.size and min(16, n) <= S.size <= min(4096, n)
        assert S.max() < n
