"""GPU parity of the two-dimensional sweep of heavy rows (edge plans of large
graphs: row blocks x neighbour slabs with both codes in LDS, partial win
counts per part summed per row afterwards).  The environment forces that path
onto small graphs with small blocks, slabs and parts, so that blocks span
many slabs, slabs hold few slots, parts cut blocks and segments, and slabs
end at the vertex count; every result must equal the oracle's exactly, as
the decisions do not depend on the sweep's layout."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import announce, check_fw

pytestmark = pytest.mark.gpu
lds = pytest.importorskip("paper_2504_10937_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

GOLD = os.path.join(os.path.dirname(__file__), "golden")

SHAPES = [
    dict(LDS_HEAVY_DEG="8", LDS_HEAVY_ROWS="64", LDS_HEAVY_SLAB="256", LDS_HEAVY_PART="128"),
    dict(LDS_HEAVY_DEG="20", LDS_HEAVY_ROWS="512", LDS_HEAVY_SLAB="1000", LDS_HEAVY_PART="4096"),
    dict(LDS_HEAVY_DEG="1", LDS_HEAVY_SLAB="1000"),  # every row heavy, one block of the default size
]
GRAPHS = [
    ("pl", dict(n=6000, beta=2.2, avg_deg=10.0, n_blocks=6, s_lo=20, s_hi=80, p_block=0.4, seed=71)),
    ("hk", dict(n=5000, mper=6, p_triad=0.6, seed=72)),
    ("small", {}),
]


def make(kind, kw):
    if kind == "pl":
        return synth.powerlaw_planted(**kw)
    if kind == "hk":
        return synth.holme_kim(**kw)
    return synth.workload("lds_small")[:3]


@pytest.fixture
def heavy_env(monkeypatch):
    def set_shape(shape):
        monkeypatch.setenv("LDS_HEAVY_MIN_SLOTS", "0")
        for k, v in shape.items():
            monkeypatch.setenv(k, v)
    return set_shape


@pytest.mark.parametrize("shape", range(len(SHAPES)))
@pytest.mark.parametrize("graph", range(len(GRAPHS)))
def test_heavy_fw_and_alg2_exact(heavy_env, shape, graph):
    heavy_env(SHAPES[shape])
    kind, kw = GRAPHS[graph]
    n, s, d = make(kind, kw)
    announce("heavy", SHAPES[shape], kind, n)
    G = oracle.Graph(n, s, d)
    g = lds.lds_create_graph(n, s, d)
    info = lds.lds_sweep_info(g, 2)
    assert info["hub_rows"] > 0, "the 2D part was not built"
    iters = 60
    _, _, out, ref = check_fw(n, s, d, 2, iters, G=G, gpu_graph=g)
    order, E, inI = lds.lds_sort_prefix(g, 2)
    o_order, o_E, o_inI = oracle.sort_prefix(G, 2, ref["A"])
    np.testing.assert_array_equal(order, o_order)
    np.testing.assert_array_equal(E, o_E)
    np.testing.assert_array_equal(inI, o_inI)
    groups, lo, hi = lds.lds_stable_groups(g, 2)
    o_groups, o_lo, o_hi = oracle.extract_sg(G, 2, ref["A"], ref["split"], ref["D"])
    assert groups == o_groups
    np.testing.assert_array_equal(lo, o_lo)
    np.testing.assert_array_equal(hi, o_hi)
    if n <= 2000:
        got = lds.lds_topk(g, 2, 5, iters)
        want = oracle.top_k(G, 2, 5)
        assert len(got) == len(want)
        for (gv, gr), (wv, wr) in zip(got, want):
            assert gr == wr
            np.testing.assert_array_equal(gv, wv)
    # the no-allocation entry point runs the same kernels
    r = torch.empty(n, dtype=torch.float32, device="cuda")
    gap = lds.lds_frank_wolfe_noalloc(g, 2, iters, r_out=r, want_gap=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.cpu().numpy(), (ref["A"].astype(np.float64) / ref["D"]).astype(np.float32))
    np.testing.assert_allclose(gap, ref["gap"], rtol=1e-12, atol=1e-12 * max(1.0, float(np.abs(ref["gap"]).max())))
    g.destroy()


def test_heavy_mid_size_golden(heavy_env):
    """The 120,000-vertex graph with every row of degree >= 32 swept in two
    dimensions (default block and slab sizes): loads, Alg. 2 order, prefix,
    I, stable groups and bounds equal the oracle's digests."""
    import hashlib
    heavy_env(dict(LDS_HEAVY_DEG="32"))
    with open(os.path.join(GOLD, "mid_size_edge.json")) as f:
        ref = json.load(f)
    n, s, d = synth.powerlaw_planted(**ref["graph"])
    announce("heavy mid size", n)
    g = lds.lds_create_graph(n, s, d)
    assert lds.lds_sweep_info(g, 2)["hub_rows"] > 0

    def sha(a, dt):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=dt).tobytes()).hexdigest()

    out = lds.lds_frank_wolfe(g, 2, ref["iters"], want_num=True, want_gap=True)
    assert sha(out["num"], "<u8") == ref["A_sha256"]
    np.testing.assert_allclose(out["gap"], ref["gap"], rtol=1e-12, atol=0.0)
    order, E, inI = lds.lds_sort_prefix(g, 2)
    assert sha(order, "<i4") == ref["order_sha256"] and sha(E, "<i8") == ref["E_sha256"]
    assert sha(inI.astype(np.uint8), "u1") == ref["inI_sha256"]
    groups, lo, hi = lds.lds_stable_groups(g, 2)
    assert len(groups) == ref["n_groups"]
    assert sha([a for a, _ in groups], "<i8") == ref["gstart_sha256"]
    assert sha(lo, "<i8") == ref["lo_sha256"] and sha(hi, "<i8") == ref["hi_sha256"]
    g.destroy()
