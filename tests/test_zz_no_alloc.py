"""cc_count_static (the counting call that allocates no device memory: its
buffers are carved from the library's static scratch) against cc_count on
the same inputs, bit for bit, on two calls in a row -- the second on a
smaller graph, so that it runs over what the first left in the scratch --
and a solve too large for the scratch is refused with CC_E_NOMEM."""
import numpy as np
import pytest

from cc_inputs import graphs, queries as Q

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1602_04478_amd.cc")


def _same(g, q, seed, trials):
    a = cc.count_static(g, q, seed, trials)
    b = cc.count(g, q, seed, trials)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2] == b[2]
    assert a[3] == b[3] or (np.isnan(a[3]) and np.isnan(b[3]))
    return a


def test_static_matches_count_two_calls():
    big = graphs.chung_lu(3000, 8.0, 2.1, None, seed=41)
    small = graphs.erdos_renyi(400, 6.0, seed=42)
    gb, gs = cc.Graph.from_csr(big), cc.Graph.from_csr(small)
    q7 = cc.Query(*Q.cycle_pendant(6))
    q5 = cc.Query(*Q.cycle(5))
    print("[no-alloc] chung-lu 3000, C6+pendant, 3 colourings", flush=True)
    a = _same(gb, q7, 11, 3)
    assert any(int(x) > 0 for x in a[0])
    print("[no-alloc] erdos-renyi 400, C5, 2 colourings", flush=True)
    _same(gs, q5, 12, 2)
    print("[no-alloc] chung-lu 3000 again, domino+tail, 2 colourings", flush=True)
    _same(gb, cc.Query(*Q.domino_tail()), 13, 2)


def test_static_refuses_what_does_not_fit():
    g = graphs.cycle_graph(4_000_000)
    dg = cc.Graph.from_csr(g)
    print("[no-alloc] cycle graph of 4e6 vertices: must not fit the scratch", flush=True)
    with pytest.raises(cc.CCError) as e:
        cc.count_static(dg, cc.Query(*Q.cycle_pendant(6)), 1, 1)
    assert e.value.name == "CC_E_NOMEM"
