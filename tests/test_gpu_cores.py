"""GPU parity of lds_core_numbers (core and tr-core numbers, the bounds of
Section 4.3 and the residual-graph numbers of Pruning rule 2, Alg. 3) with
the oracle's core numbers by their definition: bit-exact, whole graph and
induced subgraphs.  At the size of the large edge workload the numbers are
checked through two properties that the exact numbers have at any size; a
value that is too large fails the first, a single value that is too small
the second."""
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


def induced(n, s, d, alive):
    """edges of the subgraph induced by alive, relabelled; -> (m, s, d, ids)"""
    ids = np.flatnonzero(alive)
    new = np.full(n, -1, np.int64)
    new[ids] = np.arange(len(ids))
    keep = alive[s] & alive[d]
    return len(ids), new[s[keep]].astype(np.int32), new[d[keep]].astype(np.int32), ids


def check(n, s, d, mode, alive=None):
    g = lds.lds_create_graph(n, s, d)
    got = lds.lds_core_numbers(g, mode, alive)
    if alive is None:
        want = oracle.core_numbers(oracle.Graph(n, s, d), mode)
    else:
        alive = np.asarray(alive, bool)
        k, ss, dd, ids = induced(n, s, d, alive)
        want = np.full(n, -1, np.int64)
        if k:
            want[ids] = oracle.core_numbers(oracle.Graph(k, ss, dd), mode)
    np.testing.assert_array_equal(got, want)
    return got


GRAPHS = {
    "lds_small": lambda: synth.workload("lds_small")[:3],
    "holme_kim_20k": lambda: synth.holme_kim(20000, 6, 0.5, seed=7),
    "erdos_renyi": lambda: synth.erdos_renyi(3000, 0.004, seed=4),
    "powerlaw_30k": lambda: synth.powerlaw_planted(30000, 2.2, 12.0, 10, 20, 150, 0.4, seed=9),
    "powerlaw_100k": lambda: synth.powerlaw_planted(100000, 2.2, 12.0, 20, 20, 300, 0.4, seed=9),
}
CASES = [(name, mode) for name in sorted(GRAPHS) for mode in (2, 3) if (name, mode) != ("powerlaw_100k", 3)]


@pytest.mark.parametrize("name,mode", CASES)
def test_whole_graph(name, mode):
    announce("core numbers", name, mode)
    n, s, d = GRAPHS[name]()
    c = check(n, s, d, mode)
    assert c.min() >= 0


@pytest.mark.parametrize("wg", ["2", "7", "64"])
@pytest.mark.parametrize("name,mode", [("holme_kim_20k", 3), ("powerlaw_30k", 2), ("powerlaw_30k", 3)])
def test_grid_widths(name, mode, wg, monkeypatch):
    """the levels with many vertices run as one cooperative launch; its
    phases and counter ring give the same numbers at any grid width"""
    monkeypatch.setenv("LDS_PEEL_WG", wg)
    announce("core numbers grid", name, mode, wg)
    n, s, d = GRAPHS[name]()
    check(n, s, d, mode)


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_induced_subgraph(mode, seed):
    announce("core numbers induced", mode, seed)
    n, s, d = synth.powerlaw_planted(20000, 2.2, 10.0, 10, 20, 120, 0.5, seed=20 + seed)
    alive = np.random.default_rng(seed).random(n) < (0.3, 0.7, 0.95)[seed]
    check(n, s, d, mode, alive)


@pytest.mark.parametrize("mode", [2, 3])
def test_degenerate(mode):
    announce("core numbers degenerate", mode)
    e = np.zeros(0, np.int32)
    # no vertices, only isolated vertices, one edge, a clique with a tail
    assert len(lds.lds_core_numbers(lds.lds_create_graph(0, e, e), mode)) == 0
    check(5, e, e, mode)
    check(2, np.array([0], np.int32), np.array([1], np.int32), mode)
    k = 9
    s = [i for i in range(k) for j in range(i + 1, k)] + [k - 1, k, k + 1]
    t = [j for i in range(k) for j in range(i + 1, k)] + [k, k + 1, k + 2]
    c = check(k + 4, np.array(s, np.int32), np.array(t, np.int32), mode)
    assert c[0] == (k - 1 if mode == 2 else (k - 1) * (k - 2) // 2)
    # everything outside, and a mask that keeps one vertex
    check(k + 4, np.array(s, np.int32), np.array(t, np.int32), mode, np.zeros(k + 4, bool))
    one = np.zeros(k + 4, bool)
    one[3] = True
    check(k + 4, np.array(s, np.int32), np.array(t, np.int32), mode, one)


def test_bad_arguments():
    g = lds.lds_create_graph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(lds.LdsError):
        lds.lds_core_numbers(g, 5)
    with pytest.raises(ValueError):
        lds.lds_core_numbers(g, 2, np.ones(2, bool))


def test_large_edge_workload_properties():
    """At n = 4M, m = 98M: for every vertex v, at least c(v) neighbours have
    c >= c(v) (so {c >= k} lies in the k-core: c never exceeds the core
    number) and at most c(v) neighbours have c > c(v) (else v would belong to
    the (c(v)+1)-core)."""
    announce("core numbers lds_large properties")
    n, s, d = synth.workload("lds_large")[:3]
    g = lds.lds_create_graph(n, s, d)
    c = lds.lds_core_numbers(g, 2)
    G = oracle.Graph(n, s, d)
    u, v = G.edges()
    del s, d
    cu, cv = c[u], c[v]
    at_least = np.bincount(u, weights=cv >= cu, minlength=n) + np.bincount(v, weights=cu >= cv, minlength=n)
    above = np.bincount(u, weights=cv > cu, minlength=n) + np.bincount(v, weights=cu > cv, minlength=n)
    assert (at_least >= c).all()
    assert (above <= c).all()
    deg = G.degrees()
    assert (c <= deg).all() and c.max() > 100
