"""GPU parity for Alg. 2 (sort, prefix counts, index set I, stable groups and
their bounds) against the CPU oracle, exact."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import announce

pytestmark = pytest.mark.gpu
lds = pytest.importorskip("paper_2504_10937_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def check_sg(n, s, d, mode, iters):
    G = oracle.Graph(n, s, d)
    g = lds.lds_create_graph(n, s, d)
    out = lds.lds_frank_wolfe(g, mode, iters, want_num=True)
    ref = oracle.fw_exact(G, mode, iters, with_gap=False)
    np.testing.assert_array_equal(out["num"], ref["A"])
    order, E, inI = lds.lds_sort_prefix(g, mode)
    o_order, o_E, o_inI = oracle.sort_prefix(G, mode, ref["A"])
    np.testing.assert_array_equal(order, o_order)
    np.testing.assert_array_equal(E, o_E)
    np.testing.assert_array_equal(inI, o_inI)
    groups, lo, hi = lds.lds_stable_groups(g, mode)
    o_groups, o_lo, o_hi = oracle.extract_sg(G, mode, ref["A"], ref["split"], ref["D"])
    assert groups == o_groups
    np.testing.assert_array_equal(lo, o_lo)
    np.testing.assert_array_equal(hi, o_hi)
    return g, groups


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("iters", [1, 5, 60, 2000])
def test_running_example(mode, iters):
    announce("sg running example", mode, iters)
    with open(os.path.join(GOLD, "running_example.json")) as f:
        d = json.load(f)
    e = np.array(d["edges"], np.int32)
    check_sg(d["n"], e[:, 0].copy(), e[:, 1].copy(), mode, iters)


@pytest.mark.parametrize("mode", [2, 3])
def test_lds_small_workload(mode):
    n, s, d, _, iters, _ = synth.workload("lds_small")
    announce("sg lds_small", mode)
    check_sg(n, s, d, mode, iters)


CASES = [
    ("pl", dict(n=3000, beta=2.1, avg_deg=16.0, n_blocks=8, s_lo=30, s_hi=120, p_block=0.3, seed=2), 2, 100),
    ("pl", dict(n=3000, beta=2.1, avg_deg=16.0, n_blocks=8, s_lo=30, s_hi=120, p_block=0.3, seed=2), 3, 60),
    ("hk", dict(n=2000, mper=8, p_triad=0.6, seed=3), 3, 200),
    ("hk", dict(n=2000, mper=8, p_triad=0.6, seed=3), 2, 30),
    ("er", dict(n=60, p=0.3, seed=4), 2, 3),
    ("er", dict(n=60, p=0.3, seed=4), 3, 3),
    ("pl", dict(n=6000, beta=2.3, avg_deg=10.0, n_blocks=3, s_lo=600, s_hi=1500, p_block=0.9, seed=7), 2, 40),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_graphs(case):
    kind, kw, mode, iters = CASES[case]
    announce("sg", kind, kw, mode, iters)
    n, s, d = synth.erdos_renyi(**kw) if kind == "er" else (
        synth.powerlaw_planted(**kw) if kind == "pl" else synth.holme_kim(**kw))
    check_sg(n, s, d, mode, iters)


# launch shapes of the scan: every phase posted to a grid of helpers, and a
# mix where the leader keeps the small phases (the defaults give one
# workgroup below 16384 vertices, so these graphs would not reach the grid)
SHAPES = [
    {"LDS_SCAN_WG": "8", "LDS_SCAN_LEAD_RECS": "0", "LDS_SCAN_LEAD_POS": "0"},
    {"LDS_SCAN_WG": "3", "LDS_SCAN_LEAD_RECS": "300", "LDS_SCAN_LEAD_POS": "200"},
    {"LDS_SCAN_WG": "2", "LDS_SCAN_LEAD_RECS": "4000", "LDS_SCAN_LEAD_POS": "1500"},
]


@pytest.mark.parametrize("shape", range(len(SHAPES)))
@pytest.mark.parametrize("case", [0, 1, 2, 6])
def test_grid_shapes(case, shape, monkeypatch):
    """the leader / helper protocol of the scan, exact against the oracle"""
    for k, v in SHAPES[shape].items():
        monkeypatch.setenv(k, v)
    kind, kw, mode, iters = CASES[case]
    announce("sg grid", SHAPES[shape], kind, kw, mode, iters)
    n, s, d = synth.erdos_renyi(**kw) if kind == "er" else (
        synth.powerlaw_planted(**kw) if kind == "pl" else synth.holme_kim(**kw))
    g, groups = check_sg(n, s, d, mode, iters)
    check_scan_info(g, mode, groups, int(SHAPES[shape]["LDS_SCAN_WG"]))


def check_scan_info(g, mode, groups, wg):
    """the scan's phase profile (lds_sg_scan_info) is consistent with its
    result and launch shape"""
    info = lds.lds_sg_scan_info(g, mode)
    assert info["groups"] == len(groups)
    assert info["rounds"] >= info["groups"] and info["rounds"] <= info["groups"] + 1
    assert info["verifications"] >= info["groups"]
    assert info["workgroups"] == wg
    for k in ("search", "update", "minmax", "accept"):
        assert 0 <= info["grid_" + k] and info["us_" + k] >= 0
    assert info["grid_update"] <= info["verifications"] and info["grid_minmax"] <= info["verifications"]
    if wg == 1:
        assert all(info["grid_" + k] == 0 for k in ("search", "update", "minmax", "accept"))
    assert info["walked"] >= 0 and info["searched"] >= 0


def test_scan_info_default_shape_and_errors():
    """below 16,384 vertices the scan is one workgroup with no grid phase;
    before any scan the profile is an error"""
    n, s, d, mode, iters, _ = synth.workload("lds_small")
    g = lds.lds_create_graph(n, s, d)
    with pytest.raises(lds.LdsError):
        lds.lds_sg_scan_info(g, mode)
    lds.lds_frank_wolfe(g, mode, iters)
    groups, _, _ = lds.lds_stable_groups(g, mode)
    check_scan_info(g, mode, groups, 1)
    g.destroy()


@pytest.mark.parametrize("mode", [2, 3])
def test_grid_shapes_lds_small(mode, monkeypatch):
    for k, v in SHAPES[1].items():
        monkeypatch.setenv(k, v)
    n, s, d, _, iters, _ = synth.workload("lds_small")
    announce("sg grid lds_small", mode)
    check_sg(n, s, d, mode, iters)


def test_empty_and_edgeless():
    for n in (0, 5):
        g = lds.lds_create_graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
        for mode in (2, 3):
            lds.lds_frank_wolfe(g, mode, 3)
            order, E, inI = lds.lds_sort_prefix(g, mode)
            assert sorted(order.tolist()) == list(range(n)) and (E == 0).all()
            groups, lo, hi = lds.lds_stable_groups(g, mode)
            G = oracle.Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
            ref = oracle.fw_exact(G, mode, 3, with_gap=False)
            o_groups, o_lo, o_hi = oracle.extract_sg(G, mode, ref["A"], ref["split"], ref["D"])
            assert groups == o_groups
            np.testing.assert_array_equal(lo, o_lo)


def test_requires_fw_state():
    g = lds.lds_create_graph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(lds.LdsError):
        lds.lds_sort_prefix(g, 2)


def test_edge_state_survives_triangle_listing():
    """Listing triangles after an edge run leaves the edge state usable: the
    edge slot order is fixed at ingest."""
    announce("sg edge state after triangle listing")
    n, s, d = synth.powerlaw_planted(1500, 2.2, 10.0, n_blocks=4, s_lo=20, s_hi=40, p_block=0.5, seed=11)
    g = lds.lds_create_graph(n, s, d)
    lds.lds_frank_wolfe(g, 2, 30)
    lds.lds_triangles(g)
    h = lds.lds_create_graph(n, s, d)
    lds.lds_frank_wolfe(h, 2, 30)
    for a, b in zip(lds.lds_splits(g, 2), lds.lds_splits(h, 2)):
        np.testing.assert_array_equal(a, b)
    ga, lo_a, hi_a = lds.lds_stable_groups(g, 2)
    gb, lo_b, hi_b = lds.lds_stable_groups(h, 2)
    assert ga == gb
    np.testing.assert_array_equal(lo_a, lo_b)
    np.testing.assert_array_equal(hi_a, hi_b)


def test_split_width_limit():
    """The stable-group pass keeps split numerators in 32 bits: a run whose
    D_N exceeds 2^32 - 1 is refused with LDS_E_OVERFLOW before any work
    (edges from N = 65535, triangles from N = 37836), and the largest N
    that fits still runs."""
    announce("split width limit")
    # K4 plus a pendant edge: triangles and edges
    s = np.array([0, 0, 0, 1, 1, 2, 3], np.int32)
    d = np.array([1, 2, 3, 2, 3, 3, 4], np.int32)
    g = lds.lds_create_graph(5, s, d)
    for mode, n_bad in ((2, 65535), (3, 37836)):
        with pytest.raises(lds.LdsError) as e:
            lds.lds_topk(g, mode, 1, n_bad)
        assert e.value.status == 4
    lds.lds_frank_wolfe(g, 3, 37836)
    with pytest.raises(lds.LdsError) as e:
        lds.lds_sort_prefix(g, 3)
    assert e.value.status == 4
    with pytest.raises(lds.LdsError) as e:
        lds.lds_stable_groups(g, 3)
    assert e.value.status == 4
    out = lds.lds_frank_wolfe(g, 3, 37835, want_num=True)
    assert lds.lds_denominator(3, 37835) <= 2**32 - 1
    order, E, inI = lds.lds_sort_prefix(g, 3)
    assert E[-1] == 4  # K4 holds the graph's four triangles
    groups, lo, hi = lds.lds_stable_groups(g, 3)
    assert len(groups) >= 1
    g.destroy()


def test_concurrent_wide_scans():
    """Two stable-group scans of graphs above 16,384 vertices (so each is a
    cooperative launch of the wide grid) run at once from two threads on two
    streams, as serving workers do; each gives what it gives alone."""
    import threading
    graphs = [synth.powerlaw_planted(40000, 2.1, 10.0, n_blocks=12, s_lo=30, s_hi=200, p_block=0.3, seed=s)
              for s in (41, 42)]
    gs, want = [], []
    for n, s, d in graphs:
        announce("concurrent scans", n)
        g = lds.lds_create_graph(n, s, d)
        lds.lds_frank_wolfe(g, 2, 60)
        want.append(lds.lds_stable_groups(g, 2))
        assert lds.lds_sg_scan_info(g, 2)["workgroups"] > 1
        gs.append(g)
    torch.cuda.synchronize()
    for rep in range(3):
        got = [None, None]
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]

        def run(i):
            got[i] = lds.lds_stable_groups(gs[i], 2, stream=streams[i])

        ts = [threading.Thread(target=run, args=(i,)) for i in range(2)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        torch.cuda.synchronize()
        for (wg, wlo, whi), (gg, glo, ghi) in zip(want, got):
            assert gg == wg
            np.testing.assert_array_equal(glo, wlo)
            np.testing.assert_array_equal(ghi, whi)
    for g in gs:
        g.destroy()
