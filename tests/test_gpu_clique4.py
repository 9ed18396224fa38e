"""GPU parity of the 4-clique program (the h-clique program that Eq. trcp
generalises, h = 4): 4-clique listing bit-exact against the oracle's
enumeration-pinned listing, and the exact Frank-Wolfe state (numerators,
splits, duality gap) against the oracle's iteration."""
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

GRAPHS = {
    "lds_small": lambda: synth.workload("lds_small")[:3],
    "erdos_renyi_dense": lambda: synth.erdos_renyi(300, 0.2, seed=3),
    "holme_kim_20k": lambda: synth.holme_kim(20000, 8, 0.7, seed=5),
    "powerlaw_30k": lambda: synth.powerlaw_planted(30000, 2.2, 10.0, 12, 20, 90, 0.5, seed=6),
}


def clique_parity(n, s, d):
    G = oracle.Graph(n, s, d)
    g = lds.lds_create_graph(n, s, d)
    Q, q, cnt = lds.lds_cliques4(g, want_list=True, want_counts=True)
    want, wcnt = oracle.cliques4(G)
    assert Q == len(want)
    np.testing.assert_array_equal(q, want)
    np.testing.assert_array_equal(cnt, wcnt)
    return g, G, Q


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_listing(name):
    announce("clique4 listing", name)
    n, s, d = GRAPHS[name]()
    _, _, Q = clique_parity(n, s, d)
    assert Q > 0


@pytest.mark.parametrize("iters", [0, 1, 7, 100])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_frank_wolfe(name, iters):
    announce("clique4 fw", name, iters)
    n, s, d = GRAPHS[name]()
    check_fw(n, s, d, lds.LDS_CLIQUE4, iters)


def test_k4_hand_iterates_and_degenerate():
    announce("clique4 degenerate")
    k4 = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    s = np.array([e[0] for e in k4], np.int32)
    t = np.array([e[1] for e in k4], np.int32)
    g = lds.lds_create_graph(4, s, t)
    for it, A in {0: [1, 1, 1, 1], 1: [1, 1, 1, 9], 2: [1, 1, 13, 9], 3: [1, 17, 13, 9]}.items():
        out = lds.lds_frank_wolfe(g, lds.LDS_CLIQUE4, it, want_num=True)
        assert out["num"].tolist() == A and out["D"] == 2 * (it + 1) * (it + 2)
    # triangles but no 4-clique; no edges at all; isolated vertices around a K4
    tri = lds.lds_create_graph(3, np.array([0, 1, 0], np.int32), np.array([1, 2, 2], np.int32))
    assert lds.lds_cliques4(tri)[0] == 0
    out = lds.lds_frank_wolfe(tri, lds.LDS_CLIQUE4, 5, want_num=True, want_gap=True)
    assert out["num"].tolist() == [0, 0, 0] and (out["gap"] == 0).all()
    e = np.zeros(0, np.int32)
    assert lds.lds_cliques4(lds.lds_create_graph(0, e, e))[0] == 0
    check_fw(10, s + 3, t + 3, lds.LDS_CLIQUE4, 4)
    # the calls that take only edges / triangles refuse the 4-clique mode
    with pytest.raises(lds.LdsError):
        lds.lds_topk(g, lds.LDS_CLIQUE4, 1, 10)
    with pytest.raises(lds.LdsError):
        lds.lds_stable_groups(g, lds.LDS_CLIQUE4)
    assert lds.lds_denominator(lds.LDS_CLIQUE4, 100) == 2 * 101 * 102


def test_modes_share_a_graph():
    """edge, triangle and 4-clique states live side by side: running one mode
    leaves the others' results unchanged"""
    announce("clique4 mixed modes")
    n, s, d = GRAPHS["holme_kim_20k"]()
    g = lds.lds_create_graph(n, s, d)
    a2 = lds.lds_frank_wolfe(g, lds.LDS_EDGE, 30, want_num=True)["num"]
    a3 = lds.lds_frank_wolfe(g, lds.LDS_TRIANGLE, 30, want_num=True)["num"]
    a4 = lds.lds_frank_wolfe(g, lds.LDS_CLIQUE4, 30, want_num=True)["num"]
    np.testing.assert_array_equal(lds.lds_loads(g, lds.LDS_EDGE, want_num=True)["num"], a2)
    np.testing.assert_array_equal(lds.lds_loads(g, lds.LDS_TRIANGLE, want_num=True)["num"], a3)
    G = oracle.Graph(n, s, d)
    np.testing.assert_array_equal(a4, oracle.fw_exact(G, 4, 30, with_gap=False, with_split=False)["A"])


def test_large_planted():
    """n = 200k power-law graph with 40 planted blocks (16M 4-cliques):
    listing and 20 exact iterations against the oracle, whole arrays"""
    announce("clique4 large planted")
    n, s, d = synth.powerlaw_planted(200000, 2.2, 10.0, 40, 20, 120, 0.5, seed=7)
    g, G, Q = clique_parity(n, s, d)
    assert Q > 10_000_000
    check_fw(n, s, d, lds.LDS_CLIQUE4, 20, G=G, gpu_graph=g)


def neighbourhood_triangles(rp, col, u):
    """4-cliques at u = triangles of the subgraph induced by N(u), counted by
    the oracle's (enumeration-pinned) triangle listing"""
    nb = col[rp[u]:rp[u + 1]]
    if len(nb) < 3:
        return 0
    loc = {int(x): i for i, x in enumerate(nb)}
    src, dst = [], []
    for x in nb:
        for y in col[rp[x]:rp[x + 1]]:
            j = loc.get(int(y))
            if j is not None and int(x) < int(y):
                src.append(loc[int(x)])
                dst.append(j)
    return len(oracle.triangles(oracle.Graph(len(nb), np.array(src, np.int32), np.array(dst, np.int32)))[0])


def test_full_size_workload_properties():
    """The 4-clique workload (n = 1M, 200 planted blocks, 1.66e8 4-cliques):
    per-vertex counts at sampled vertices from the triangles of their
    neighbourhoods; sum of counts = 4 Q; after 100 iterations every numerator
    is q_u plus multiples of 4 (a0 = 1, increments 4(i+1)), they sum to D Q,
    and the gap is non-negative and falls."""
    announce("clique4 full-size properties")
    n, s, d, mode, iters, _ = synth.workload("clique4_pl")
    g = lds.lds_create_graph(n, s, d)
    Q, _, cnt = lds.lds_cliques4(g, want_counts=True)
    assert int(cnt.sum()) == 4 * Q and Q > 100_000_000
    G = oracle.Graph(n, s, d)
    u, v = G.edges()
    del s, d
    order = np.argsort(np.concatenate([u, v]), kind="stable")
    col = np.concatenate([v, u])[order]
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(np.concatenate([u, v]), minlength=n), out=rp[1:])
    deg = np.diff(rp)
    rng = np.random.default_rng(5)
    sample = np.concatenate([rng.choice(np.flatnonzero((deg >= 3) & (deg <= 400)), 60, replace=False),
                             rng.choice(np.flatnonzero(cnt > 1000), 20, replace=False)])
    for x in sample:
        if deg[x] <= 400:
            assert neighbourhood_triangles(rp, col, x) == cnt[x], x
    out = lds.lds_frank_wolfe(g, mode, iters, want_num=True, want_gap=True)
    A = out["num"].astype(np.int64)
    assert ((A - cnt) % 4 == 0).all() and (A >= cnt).all()
    assert int(out["num"].sum(dtype=np.uint64)) == out["D"] * Q
    gap = out["gap"]
    assert (gap >= 0).all() and gap[-1] < gap[0]
