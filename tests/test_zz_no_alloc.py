"""The entry point that allocates nothing (bc_brandes_plain_noalloc), through the C-ABI,
against the allocating one (bc_brandes_plain_dev) on the same inputs: two calls in a
row, the second with a smaller graph and fewer targets. Scores agree within 1e-9
relative (exact zeros where the other has zeros); the small call also matches the
oracle. The first call is large enough to run its source groups in several waves
through the fixed scratch array. A call on a fresh graph handle leaves the device's
free memory unchanged."""
import numpy as np
import pytest

import oracle
from paper_1406_4173_amd import inputs

pytestmark = pytest.mark.gpu

REL = 1e-9


def close(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    assert np.array_equal(got == 0, want == 0), "zero pattern differs"
    err = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
    err[want == 0] = 0
    assert err.max(initial=0) <= REL, f"max rel err {err.max()}"


def test_noalloc_matches_allocating_entry_point_twice():
    import torch

    from paper_1406_4173_amd import bcpp

    bcpp.lib()
    dev = torch.device("cuda:0")
    cases = []
    g = inputs.pareto_100k()
    cases.append((g, g.S[:600]))
    g = inputs.planted_1k()
    cases.append((g, inputs.random_targets(17, g.n, 300)))
    for i, (g, S) in enumerate(cases):
        print(f"no-alloc call {i}: n={g.n} |S|={len(S)}", flush=True)
        G = bcpp.Graph(g, stream=torch.cuda.current_stream(dev))
        S_dev = torch.tensor(np.asarray(S, np.int32), device=dev)
        want = torch.empty(g.n, dtype=torch.float64, device=dev)
        got = torch.full((g.n,), -1.0, dtype=torch.float64, device=dev)
        bcpp.brandes_plain_noalloc(G, S_dev, got)
        bcpp.brandes_plain_dev(G, S_dev, want)
        torch.cuda.synchronize()
        close(got.cpu().numpy(), want.cpu().numpy())
        if i == 1:
            close(got.cpu().numpy(), oracle.bc(g, np.asarray(S)))
        got2 = torch.full((g.n,), -1.0, dtype=torch.float64, device=dev)
        bcpp.brandes_plain_noalloc(G, S_dev, got2, ordered=True)
        torch.cuda.synchronize()
        close(got2.cpu().numpy(), 2 * want.cpu().numpy())


def test_noalloc_keeps_free_memory_and_rejects_too_large():
    import torch

    from paper_1406_4173_amd import bcpp

    dev = torch.device("cuda:0")
    g = inputs.planted_1k()
    S = inputs.random_targets(18, g.n, 200)
    S_dev = torch.tensor(S, device=dev)
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    bcpp.brandes_plain_noalloc(bcpp.Graph(g), S_dev, out)  # first call on the device
    torch.cuda.synchronize()
    G = bcpp.Graph(g)
    free0 = torch.cuda.mem_get_info()[0]
    bcpp.brandes_plain_noalloc(G, S_dev, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    close(out.cpu().numpy(), oracle.bc(g, S))
    # one group over a graph whose per-group buffers exceed the scratch array
    assert bcpp.noalloc_scratch_bytes() == 256 << 20
    big = inputs.path(12_000_000)
    Gb = bcpp.Graph(big)
    outb = torch.empty(big.n, dtype=torch.float64, device=dev)
    with pytest.raises(bcpp.BcError) as ei:
        bcpp.brandes_plain_noalloc(Gb, torch.tensor([0, 5], dtype=torch.int32, device=dev), outb)
    assert ei.value.code == bcpp.BC_E_NOMEM
