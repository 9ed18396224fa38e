"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: exact comparison with the oracle for the first iterations on the whole
graph (the oracle finishes those in seconds), and properties that hold at any
size for the full iteration counts."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import announce

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
lds = pytest.importorskip("paper_2504_10937_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)


def check_properties(g, mode, iters, n, P):
    D = lds.lds_denominator(mode, iters)
    r = torch.empty(n, dtype=torch.float32, device="cuda")
    out = lds.lds_frank_wolfe(g, mode, iters, r_out=r, want_num=True, want_gap=True)
    num = out["num"]
    # feasibility (Eq. cp / trcp): every pattern's unit is split, sum r = |P|
    assert int(num.sum(dtype=np.uint64)) == D * P
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.cpu().numpy(), (num.astype(np.float64) / D).astype(np.float32))
    gap = out["gap"]
    assert (gap >= 0).all()
    order, E, inI = lds.lds_sort_prefix(g, mode)
    assert np.array_equal(np.sort(order), np.arange(n))
    A = num[order]
    assert (A[:-1] >= A[1:]).all()
    ties = A[:-1] == A[1:]
    assert (order[:-1][ties] < order[1:][ties]).all()
    assert (np.diff(E) >= 0).all() and E[-1] == P and inI[-1]
    groups, lo, hi = lds.lds_stable_groups(g, mode)
    assert len(groups) > 0 and groups[0][0] == 0
    ends = set((np.flatnonzero(inI) + 1).tolist())
    prev_lo = None
    for (a, b), nxt in zip(groups, groups[1:] + [None]):
        assert b in ends
        if nxt is not None:
            assert nxt[0] == b
        vs = order[a:b]
        assert (lo[vs] == lo[vs[0]]).all() and (hi[vs] == hi[vs[0]]).all()
        assert 0 <= lo[vs[0]] <= hi[vs[0]]
        if prev_lo is not None:
            assert hi[vs[0]] < prev_lo
        prev_lo = lo[vs[0]]
    tail = order[groups[-1][1]:]
    assert (lo[tail] == -1).all() and (hi[tail] == -1).all()
    return groups


def test_lds_large_full_size():
    n, s, d, mode, iters, _ = synth.workload("lds_large")
    announce("lds_large full size", n, len(s))
    g = lds.lds_create_graph(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    G = oracle.Graph(n, s, d)
    assert lds.lds_graph_info(g)["m"] == G.m
    # exact: the first iterations over the whole graph
    N0 = 3
    out = lds.lds_frank_wolfe(g, mode, N0, want_num=True, want_gap=True)
    ref = oracle.fw_exact(G, mode, N0, with_split=False)
    np.testing.assert_array_equal(out["num"], ref["A"])
    np.testing.assert_allclose(out["gap"], ref["gap"], rtol=1e-12)
    order, E, inI = lds.lds_sort_prefix(g, mode)
    o_order, o_E, o_inI = oracle.sort_prefix(G, mode, ref["A"])
    np.testing.assert_array_equal(order, o_order)
    np.testing.assert_array_equal(E, o_E)
    np.testing.assert_array_equal(inI, o_inI)
    # the benchmark iteration count: properties
    announce("lds_large N", iters)
    check_properties(g, mode, iters, n, G.m)


def test_ltds_hk_full_size():
    n, s, d, mode, iters, _ = synth.workload("ltds_hk")
    announce("ltds_hk full size", n, len(s))
    g = lds.lds_create_graph(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    G = oracle.Graph(n, s, d)
    T, tri, cnt = lds.lds_triangles(g, want_list=True, want_counts=True)
    o_tri, o_cnt = oracle.triangles(G)
    assert T == len(o_tri)
    np.testing.assert_array_equal(tri, o_tri)
    np.testing.assert_array_equal(cnt, o_cnt)
    del tri, o_tri
    N0 = 2
    out = lds.lds_frank_wolfe(g, mode, N0, want_num=True, want_gap=True)
    ref = oracle.fw_exact(G, mode, N0, with_split=False)
    np.testing.assert_array_equal(out["num"], ref["A"])
    np.testing.assert_allclose(out["gap"], ref["gap"], rtol=1e-12)
    order, E, inI = lds.lds_sort_prefix(g, mode)
    o_order, o_E, o_inI = oracle.sort_prefix(G, mode, ref["A"])
    np.testing.assert_array_equal(order, o_order)
    np.testing.assert_array_equal(E, o_E)
    np.testing.assert_array_equal(inI, o_inI)
    announce("ltds_hk N", iters)
    check_properties(g, mode, iters, n, T)
