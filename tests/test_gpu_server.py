"""GPU tests of the served form: continuous batching of Brandes++ queries.

Every query's scores must match the oracle within 1e-9 and be identical to the same
query run alone through bc_partition_sk + bc_brandes_pp; a failing query reports its
error on poll without affecting the others.
"""
import time

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


def wait_all(srv, tickets, ns, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            try:
                r = srv.poll(t, ns[t])
            except Exception as e:  # a failed query reports its error here
                out[t] = e
                continue
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "queries did not finish"
        time.sleep(0.002)
    return out


def pool():
    gs = [inputs.random_graph(8100 + i, 60 + 15 * i, 0.06, wmax=[None, 5][i % 2], k=4 + i)
          for i in range(4)]
    gs.append(inputs.planted_1k())
    # 20,000 nodes with 15,000 cut edges: its skeletons have more nodes than LDS holds,
    # so its queries run on the engine while the others take the resident kernel
    big = inputs.sbm(inputs.rng_for(inputs.SEED_BASE + 96, 0), inputs.equal_sizes(20000, 40),
                     4.0 / 499, 15000, 3, "big20k")
    gs.append(big)
    return gs


@PATHS
def test_server_queries_match_oracle_and_alone(bcpp, engine_only):
    gs = pool()
    srv = bcpp.Server(2 << 30, max_inflight=8)
    gids = [srv.add_graph(g) for g in gs]
    rng = np.random.default_rng(5)
    queries = []
    for j in range(40):
        gi = int(rng.integers(0, len(gs)))
        g = gs[gi]
        ns = int(rng.integers(0, min(g.n, 90)))
        S = inputs.random_targets(300 + j, g.n, ns)
        queries.append((gi, S))
    tickets, ns = [], {}
    for gi, S in queries:
        t = srv.submit(gids[gi], S, engine_only=engine_only)
        tickets.append(t)
        ns[t] = gs[gi].n
    res = wait_all(srv, tickets, ns)
    for (gi, S), t in zip(queries, tickets):
        g = gs[gi]
        got = res[t]
        assert not isinstance(got, Exception), got
        assert_scores(got, oracle.bc(g, S))
        G = bcpp.Graph(g)
        alone = bcpp.brandes_pp(G, bcpp.partition_sk(G, g.part, g.k, S), engine_only=engine_only)
        assert np.array_equal(got, alone)
    st = srv.stats()
    assert st["completed"] == len(queries) and st["failed"] == 0
    assert st["p99_ms"] >= st["p50_ms"] > 0
    srv.close()


def test_server_failure_is_isolated(bcpp):
    srv = bcpp.Server(1 << 30, max_inflight=4)
    grid = inputs.grid(35, 35)
    grid.part = (np.arange(grid.n) // 35 // 5).astype(np.int32)
    grid.k = 7
    g2 = inputs.planted_1k()
    a = srv.add_graph(grid)
    b = srv.add_graph(g2)
    S2 = inputs.random_targets(9, g2.n, 50)
    t_bad = srv.submit(a, np.array([0, grid.n - 1], np.int32))
    t_good = srv.submit(b, S2)
    res = wait_all(srv, [t_bad, t_good], {t_bad: grid.n, t_good: g2.n})
    assert isinstance(res[t_bad], bcpp.BcError) and res[t_bad].code == bcpp.BC_E_OVERFLOW
    assert_scores(res[t_good], oracle.bc(g2, S2))
    with pytest.raises(bcpp.BcError) as ei:
        srv.poll(987654321, 10)
    assert ei.value.code == bcpp.BC_E_NOTFOUND
    srv.close()


def test_server_budget_too_small_for_a_query(bcpp):
    srv = bcpp.Server(64 << 20, max_inflight=2)
    g = inputs.pareto_100k()
    small = inputs.random_graph(8300, 50, 0.1, wmax=3, k=3)
    gid = srv.add_graph(g)
    sid = srv.add_graph(small)
    # 2,000 sources over a 74,000-node skeleton: hundreds of MB of per-group state
    t_big = srv.submit(gid, g.S)
    t_small = srv.submit(sid, small.S)
    res = wait_all(srv, [t_big, t_small], {t_big: g.n, t_small: small.n})
    assert isinstance(res[t_big], bcpp.BcError) and res[t_big].code == bcpp.BC_E_NOMEM
    assert_scores(res[t_small], oracle.bc(small, small.S))
    srv.close()
