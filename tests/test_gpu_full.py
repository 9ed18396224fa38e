"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: exact comparison with the oracle for the first iterations on the whole
graph (the oracle finishes those in seconds); at the full iteration counts,
properties that hold at any size and the oracle's own results stored by
tests/golden/make_full_size.py (exact loads, gap, Alg. 2's order, prefix
counts and index set, and the LDS / LTDS sets above the density the oracle
certifies); and Alg. 2 exactly, stable groups and bounds included, on a
120,000-vertex graph in both modes (tests/golden/make_mid_size.py)."""
import hashlib
import json
import os
from fractions import Fraction

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

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def golden(file, name=None):
    with open(os.path.join(GOLD, file)) as f:
        d = json.load(f)
    return d[name] if name else d


def check_golden_fw(out, order, E, inI, ref):
    """the library's loads after the full N and Alg. 2's sort and prefix step
    against the oracle's, stored by tests/golden/make_*_size.py"""
    assert out["D"] == ref["D"]
    if "A_sum" in ref:
        assert int(out["num"].sum(dtype=np.uint64)) == ref["A_sum"]
    assert sha(out["num"], "<u8") == ref["A_sha256"], "exact loads differ from the oracle's"
    np.testing.assert_allclose(out["gap"], ref["gap"], rtol=1e-12, atol=0.0)
    assert int(inI.sum()) == ref["n_I"]
    assert sha(order, "<i4") == ref["order_sha256"]
    assert sha(E, "<i8") == ref["E_sha256"]
    assert sha(inI.astype(np.uint8), "u1") == ref["inI_sha256"]


def check_golden_topk(g, ref):
    """the library's LDS (LTDS) sets of density >= lambda against the sets the
    oracle certified (k-core, superlevel min cut, decomposition of the
    superlevel set)"""
    lam = Fraction(*ref["lambda"])
    got = lds.lds_topk(g, ref["mode"], max(10, len(ref["sets"]) + 1), ref["iters"])
    mine = [(v, r) for v, r in got if r >= lam]
    assert len(mine) == len(ref["sets"])
    for (v, r), w in zip(mine, ref["sets"]):
        assert r == Fraction(*w["rho"])
        np.testing.assert_array_equal(v, np.array(w["vertices"], np.int32))


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
    props = (out, order, E, inI)
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
    return props


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
    # the benchmark iteration count: properties, and the oracle's exact
    # result stored as digests
    announce("lds_large N", iters)
    del G
    ref = golden("full_size.json", "lds_large")
    assert (ref["n"], ref["m"], ref["iters"]) == (n, lds.lds_graph_info(g)["m"], iters)
    check_golden_fw(*check_properties(g, mode, iters, n, ref["m"]), ref)
    announce("lds_large top-k")
    check_golden_topk(g, ref)


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
    del G
    ref = golden("full_size.json", "ltds_hk")
    assert (ref["n"], ref["patterns"], ref["iters"]) == (n, T, iters)
    check_golden_fw(*check_properties(g, mode, iters, n, T), ref)
    announce("ltds_hk top-k")
    check_golden_topk(g, ref)


@pytest.mark.parametrize("which", ["edge", "triangle"])
def test_mid_size_exact_alg2(which):
    """120,000 vertices: the codes of about a third of them (internal ids >=
    77,824) are gathered from memory, and the stable-group scan runs in its
    default multi-workgroup shape; loads, order, prefix, I, groups and bounds exactly as the oracle's
    literal Alg. 2 (digests from tests/golden/make_mid_size.py)."""
    ref = golden("mid_size_%s.json" % which)
    n, s, d = synth.powerlaw_planted(**ref["graph"])
    mode, iters = ref["mode"], ref["iters"]
    announce("mid size", which, n, iters)
    g = lds.lds_create_graph(n, s, d)
    assert lds.lds_graph_info(g)["m"] == ref["m"]
    out = lds.lds_frank_wolfe(g, mode, iters, want_num=True, want_gap=True)
    order, E, inI = lds.lds_sort_prefix(g, mode)
    check_golden_fw(out, order, E, inI, ref)
    groups, lo, hi = lds.lds_stable_groups(g, mode)
    assert len(groups) == ref["n_groups"]
    assert [list(x) for x in groups[:20]] == ref["first_groups"]
    assert sha([a for a, _ in groups], "<i8") == ref["gstart_sha256"]
    assert sha([b for _, b in groups], "<i8") == ref["gend_sha256"]
    assert sha(lo, "<i8") == ref["lo_sha256"] and sha(hi, "<i8") == ref["hi_sha256"]
    g.destroy()
