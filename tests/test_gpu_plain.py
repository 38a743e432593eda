"""GPU parity of the Brandes subroutine and plain target-set Brandes against the oracle.

Distances and path counts must match bit for bit; scores within a relative 1e-9
(plus exact zeros where the oracle has zeros).
"""
import numpy as np
import pytest

import oracle
from paper_1406_4173_amd import inputs

pytestmark = pytest.mark.gpu

REL = 1e-9
# the two traversal paths: LDS-resident kernel where the graph fits, and the engine
PATHS = pytest.mark.parametrize("engine_only", [False, True], ids=["resident", "engine"])


def assert_scores(got, want, rel=REL):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape
    assert np.array_equal(got == 0, want == 0), "zero pattern differs"
    err = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
    err[want == 0] = 0
    assert err.max(initial=0) <= rel, f"max rel err {err.max()} at {int(err.argmax())}"


@pytest.fixture(scope="module")
def bcpp():
    from paper_1406_4173_amd import bcpp as b

    b.lib()
    return b


def check_counts(b, g, src):
    G = b.Graph(g)
    d, sig = b.sssp_counts(G, src)
    for i, s in enumerate(src):
        od, osig = oracle.sssp(g, int(s))
        assert np.array_equal(d[i], od), f"distances differ from source {s}"
        assert np.array_equal(sig[i], osig), f"path counts differ from source {s}"


def test_counts_small_random(bcpp):
    for seed in range(40):
        g = inputs.random_graph(seed, 5 + seed % 20, 0.3, wmax=[None, 4][seed % 2])
        check_counts(bcpp, g, np.arange(g.n))


def test_counts_grid_and_ragged_source_counts(bcpp):
    g = inputs.grid(9, 13)
    for ns in (1, 63, 64, 65, 117):
        src = np.arange(ns) % g.n
        check_counts(bcpp, g, src)


def test_counts_planted_and_weighted(bcpp):
    g = inputs.planted_1k()
    check_counts(bcpp, g, inputs.random_targets(11, g.n, 130))
    g = inputs.sbm_10k()
    check_counts(bcpp, g, inputs.random_targets(12, g.n, 70))


def test_counts_overflow_boundary(bcpp):
    g = inputs.grid(34, 35)
    check_counts(bcpp, g, [0, g.n - 1, 17])
    g = inputs.grid(35, 35)
    G = bcpp.Graph(g)
    with pytest.raises(bcpp.BcError) as ei:
        bcpp.sssp_counts(G, [0])
    assert ei.value.code == bcpp.BC_E_OVERFLOW


@PATHS
def test_plain_small_random_graphs(bcpp, engine_only):
    for seed in range(120):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 40))
        g = inputs.random_graph(2000 + seed, n, float(rng.choice([0.05, 0.15, 0.4])),
                                wmax=[None, 3, 9][seed % 3])
        G = bcpp.Graph(g)
        for ordered in (False, True):
            assert_scores(bcpp.brandes_plain(G, g.S, ordered, engine_only=engine_only),
                          oracle.bc(g, g.S, ordered))


@PATHS
@pytest.mark.parametrize("n", [2, 7, 64, 65, 200, 3000])
def test_plain_closed_forms(bcpp, n, engine_only):
    def run(g, S):
        return bcpp.brandes_plain(bcpp.Graph(g), S, engine_only=engine_only)

    g = inputs.star(n)
    C = run(g, np.arange(n))
    assert C[0] == (n - 1) * (n - 2) / 2 and np.all(C[1:] == 0)
    g = inputs.path(n)
    i = np.arange(n)
    assert_scores(run(g, i), (i * (n - 1 - i)).astype(float))
    if n >= 3:
        g = inputs.cycle(n)
        want = (n - 2) ** 2 / 8 if n % 2 == 0 else (n - 1) * (n - 3) / 8
        assert_scores(run(g, np.arange(n)), np.full(n, want))
        g = inputs.complete(min(n, 40))
        assert np.all(run(g, np.arange(g.n)) == 0)


@PATHS
def test_plain_degenerate_target_sets(bcpp, engine_only):
    g = inputs.planted_1k()
    G = bcpp.Graph(g)
    for S in ([], [3]):
        assert np.all(bcpp.brandes_plain(G, np.array(S, np.int32), engine_only=engine_only) == 0)
    S = [5, 900]
    assert_scores(bcpp.brandes_plain(G, S, engine_only=engine_only), oracle.bc(g, np.array(S)))
    with pytest.raises(bcpp.BcError):
        bcpp.brandes_plain(G, [1, 1])
    with pytest.raises(bcpp.BcError):
        bcpp.brandes_plain(G, [1, g.n])
    e = inputs.empty(10)
    assert np.all(bcpp.brandes_plain(bcpp.Graph(e), np.arange(10), engine_only=engine_only) == 0)


@PATHS
def test_plain_overflow(bcpp, engine_only):
    g = inputs.grid(35, 35)
    with pytest.raises(bcpp.BcError) as ei:
        bcpp.brandes_plain(bcpp.Graph(g), [0, g.n - 1], engine_only=engine_only)
    assert ei.value.code == bcpp.BC_E_OVERFLOW
    g = inputs.grid(34, 35)
    assert_scores(bcpp.brandes_plain(bcpp.Graph(g), [0, g.n - 1], engine_only=engine_only),
                  oracle.bc(g, np.array([0, g.n - 1])))


@PATHS
def test_plain_planted_1k_full(bcpp, engine_only):
    g = inputs.planted_1k()
    assert_scores(bcpp.brandes_plain(bcpp.Graph(g), g.S, engine_only=engine_only), oracle.bc(g, g.S))


@PATHS
def test_plain_sbm_10k_full(bcpp, engine_only):
    g = inputs.sbm_10k()
    assert_scores(bcpp.brandes_plain(bcpp.Graph(g), g.S, engine_only=engine_only), oracle.bc(g, g.S))


def test_plain_resident_overflow_in_a_later_source(bcpp):
    # the overflowing source is not the first of its group: the flag must survive the
    # sources after it
    # (more than 1024 targets: two per group; corner 0 is the second source of the
    # first group, and the opposite corner is the second of the last full group)
    g = inputs.grid(35, 35)
    S = np.arange(g.n, dtype=np.int32)
    S[0], S[1] = 1, 0
    S[-1], S[-2] = S[-2], S[-1]
    for engine_only in (False, True):
        with pytest.raises(bcpp.BcError) as ei:
            bcpp.brandes_plain(bcpp.Graph(g), S, engine_only=engine_only)
        assert ei.value.code == bcpp.BC_E_OVERFLOW


def test_plain_dev_entry_point(bcpp):
    torch = pytest.importorskip("torch")
    g = inputs.planted_1k()
    G = bcpp.Graph(g)
    S = inputs.random_targets(5, g.n, 150)
    S_dev = torch.tensor(S, dtype=torch.int32, device="cuda")
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    bcpp.brandes_plain_dev(G, S_dev, out)
    torch.cuda.synchronize()
    assert_scores(out.cpu().numpy(), oracle.bc(g, S))


@pytest.mark.parametrize("n,wmax,intra", [(20000, None, 0.9), (20000, 4, 0.99), (20000, 12, 0.95),
                                           (20000, 100, 0.95)],
                         ids=["unit", "w4-chain", "w12", "w100-no-buckets"])
def test_plain_bucket_and_scan_steps_agree(bcpp, monkeypatch, n, wmax, intra):
    """A range too large for LDS keeps bucket bitmaps of the pending distances (arcs up
    to 63 long): a step with few bits reads its bucket, a dense one scans the range.
    Both queue the same nodes in the same order, so every threshold (0: always the
    bucket, 63: always the scan) gives the same bits, and those match the oracle."""
    rng = inputs.rng_for(inputs.SEED_BASE + 91, 0 if wmax is None else wmax, n)
    g = inputs._community_graph(rng, n, n // 50, 8.0, intra, wmax, "bucket")
    S = np.sort(rng.choice(g.n, 160, replace=False)).astype(np.int32)
    G = bcpp.Graph(g)
    got = {}
    for shift in ("0", "63", None):
        if shift is None:
            monkeypatch.delenv("BCPP_TUNE_DENSE_SHIFT", raising=False)
        else:
            monkeypatch.setenv("BCPP_TUNE_DENSE_SHIFT", shift)
        got[shift] = bcpp.brandes_plain(G, S)
    assert np.array_equal(got["0"], got["63"])
    assert np.array_equal(got["0"], got[None])
    assert_scores(got[None], oracle.bc(g, S))


@pytest.mark.gpu
@pytest.mark.parametrize("n,deg", [(8000, 10.0), (12000, 30.0)])
def test_plain_lds_state_with_and_without_tight_bitmap(bcpp, n, deg):
    """With the state in LDS the backward expands only the arcs that the forward found
    tight (a bitmap of the range's arcs beside the state). 8,000 nodes of degree 10
    leave room for it; 12,000 nodes of degree 30 fill LDS with the state alone (144 KB
    against 45 KB of bitmap), so every arc is tested there. Both match the oracle."""
    rng = inputs.rng_for(inputs.SEED_BASE + 93, n, int(deg))
    g = inputs._community_graph(rng, n, n // 50, deg, 0.9, 10, "tight")
    S = np.sort(rng.choice(g.n, 40, replace=False)).astype(np.int32)
    G = bcpp.Graph(g)
    assert_scores(bcpp.brandes_plain(G, S), oracle.bc(g, S))


@pytest.mark.gpu
def test_plain_lds_state_tight_bitmap_with_hubs(bcpp):
    """Nodes whose arcs span more than two words of the tight-arc bitmap count and
    select their bits in the bitmap itself rather than in registers: a 3,000-node
    community graph (state in LDS) with 5 hubs of degree 400, weights 1..3."""
    rng = inputs.rng_for(inputs.SEED_BASE + 97)
    base = inputs._community_graph(rng, 3000, 60, 8.0, 0.9, 3, "hubs")
    u, v, w = base.edges()
    hubs = np.arange(5) * 600
    hu = np.repeat(hubs, 400)
    hv = rng.choice(3000, hu.size)
    g = inputs.graph_from_edges(3000, np.concatenate([u, hu]), np.concatenate([v, hv]),
                                np.concatenate([w, rng.integers(1, 4, hu.size)]), name="hubs")
    deg = np.diff(g.row_ptr)
    assert deg[hubs].min() > 300 and g.nnz >= 6 * g.n
    S = np.union1d(hubs, rng.choice(3000, 60, replace=False)).astype(np.int32)
    G = bcpp.Graph(g)
    assert_scores(bcpp.brandes_plain(G, S), oracle.bc(g, S))
