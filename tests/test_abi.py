"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol, and
rejects malformed input on the host before any device work."""
import numpy as np
import pytest

from paper_1406_4173_amd import bcpp, inputs


def test_library_exports_every_declared_symbol():
    L = bcpp.lib()
    names = bcpp.exported_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name


def _bad_graphs():
    g = inputs.path(4)
    out = []
    b = inputs.path(4); b.col = b.col.copy(); b.col[0] = 0              # self-loop
    out.append(("self-loop", b))
    b = inputs.path(4); b.col = b.col.copy(); b.col[1] = 5              # out of range
    out.append(("range", b))
    b = inputs.path(4, w=np.array([1, 2, 3])); b.w = b.w.copy(); b.w[0] = 0   # zero weight
    out.append(("zero weight", b))
    b = inputs.path(4, w=np.array([1, 2, 3])); b.w = b.w.copy(); b.w[0] = 7   # asymmetric w
    out.append(("asym weight", b))
    # asymmetric structure: drop one arc
    rp = np.array([0, 1, 2, 2], np.int64); col = np.array([1, 2], np.int32)
    out.append(("asym", inputs.Graph(n=3, row_ptr=rp, col=col, w=None)))
    # duplicate arc
    rp = np.array([0, 2, 4], np.int64); col = np.array([1, 1, 0, 0], np.int32)
    out.append(("dup", inputs.Graph(n=2, row_ptr=rp, col=col, w=None)))
    # unsorted row_ptr
    rp = np.array([0, 2, 1, 2], np.int64); col = np.array([1, 2], np.int32)
    out.append(("row_ptr", inputs.Graph(n=3, row_ptr=rp, col=col, w=None)))
    # weight sum bound
    b = inputs.path(3, w=np.array([2 ** 30, 2 ** 30]))
    out.append(("weight bound", b))
    return out


@pytest.mark.parametrize("name,g", _bad_graphs(), ids=[n for n, _ in _bad_graphs()])
def test_invalid_graph_rejected(name, g):
    with pytest.raises(bcpp.BcError) as ei:
        bcpp.Graph(g)
    assert ei.value.code == bcpp.BC_E_INVAL
