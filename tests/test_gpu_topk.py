"""GPU parity of lds_topk (Alg. 5, LDScvx / LTDScvx) with the oracle's
top-k by the definitions: the same vertex sets, the same exact densities,
the same order.  The library's answer does not depend on the FW iteration
count (only its speed does), so several counts are checked."""
import json
import os
from fractions import Fraction

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


def same(got, ref):
    assert len(got) == len(ref), (len(got), len(ref))
    for (gv, gr), (rv, rr) in zip(got, ref):
        assert gr == rr
        np.testing.assert_array_equal(gv, rv)


def check(n, s, d, mode, k, iters, G=None):
    G = G or oracle.Graph(n, s, d)
    ref = oracle.top_k(G, mode, k)
    g = lds.lds_create_graph(n, s, d)
    got, st = lds.lds_topk(g, mode, k, iters, with_stats=True)
    same(got, ref)
    return got, st


def running_example():
    with open(os.path.join(GOLD, "running_example.json")) as f:
        d = json.load(f)
    e = np.array(d["edges"], np.int32)
    return d, d["n"], e[:, 0].copy(), e[:, 1].copy()


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("iters", [0, 1, 20, 200])
def test_running_example(mode, iters):
    announce("topk running example", mode, iters)
    d, n, s, t = running_example()
    got, _ = check(n, s, t, mode, 2, iters)
    key = "lds" if mode == 2 else "ltds"
    # the worked example's two answers (S1 and S2), densest first
    want = [(np.array(sorted(v), np.int32), Fraction(a, b)) for v, (a, b) in d[key]][:2]
    same(got, want)


@pytest.mark.parametrize("mode", [2, 3])
def test_running_example_all(mode):
    announce("topk running example all", mode)
    _, n, s, t = running_example()
    check(n, s, t, mode, 100, 50)


@pytest.mark.parametrize("mode", [2, 3])
def test_lds_small_workload(mode):
    n, s, d, _, iters, k = synth.workload("lds_small")
    announce("topk lds_small", mode, k)
    check(n, s, d, mode, k, iters)


@pytest.mark.parametrize("index", range(6))
@pytest.mark.parametrize("mode", [2, 3])
def test_batch_members(index, mode):
    n, s, d = synth.batch_member(index)
    announce("topk batch member", index, mode, n)
    check(n, s, d, mode, 10, 100 if mode == 2 else 200)


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("k", [1, 3, 1000])
def test_holme_kim(mode, k):
    n, s, d = synth.holme_kim(3000, 5, 0.6, seed=4)
    announce("topk holme-kim", mode, k)
    check(n, s, d, mode, k, 100)


@pytest.mark.parametrize("mode", [2, 3])
def test_powerlaw_planted_all_sets(mode):
    n, s, d = synth.powerlaw_planted(4000, 2.2, 10.0, n_blocks=12, s_lo=15, s_hi=80, p_block=0.4, seed=7)
    announce("topk powerlaw all", mode)
    check(n, s, d, mode, 100000, 60)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("mode", [2, 3])
def test_tiny_against_brute_force(seed, mode):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(4, 13))
    n, s, d = synth.erdos_renyi(n, float(rng.uniform(0.25, 0.7)), seed=200 + seed)
    announce("topk tiny", seed, mode, n, len(s))
    G = oracle.Graph(n, s, d)
    _, sets = oracle.brute(G, mode)
    g = lds.lds_create_graph(n, s, d)
    got = lds.lds_topk(g, mode, 1000, 10)
    same(got, sets)


@pytest.mark.parametrize("mode", [2, 3])
def test_degenerate_graphs(mode):
    announce("topk degenerate", mode)
    e = np.zeros(0, np.int32)
    g = lds.lds_create_graph(5, e, e)
    assert lds.lds_topk(g, mode, 3, 10) == []
    g = lds.lds_create_graph(0, e, e)
    assert lds.lds_topk(g, mode, 3, 10) == []
    # one edge; one triangle plus a pendant edge
    g = lds.lds_create_graph(3, np.array([2], np.int32), np.array([0], np.int32))
    got = lds.lds_topk(g, mode, 3, 10)
    if mode == 2:
        same(got, [(np.array([0, 2], np.int32), Fraction(1, 2))])
    else:
        assert got == []
    g = lds.lds_create_graph(4, np.array([0, 1, 2, 2], np.int32), np.array([1, 2, 0, 3], np.int32))
    got = lds.lds_topk(g, mode, 3, 10)
    if mode == 2:
        # the pendant vertex keeps density 1 and the whole graph is 1-compact
        same(got, [(np.array([0, 1, 2, 3], np.int32), Fraction(1))])
    else:
        same(got, [(np.array([0, 1, 2], np.int32), Fraction(1, 3))])


def test_invalid_arguments():
    announce("topk invalid")
    _, n, s, t = running_example()
    g = lds.lds_create_graph(n, s, t)
    for args in [(2, 0, 10), (2, 3, -1), (4, 3, 10)]:
        with pytest.raises(lds.LdsError) as ei:
            lds.lds_topk(g, *args)
        assert ei.value.status == 1


def test_fw_state_after_topk():
    """lds_topk leaves the graph's FW state as an iters-iteration run."""
    announce("topk fw state")
    _, n, s, t = running_example()
    g = lds.lds_create_graph(n, s, t)
    lds.lds_topk(g, 2, 2, 30)
    G = oracle.Graph(n, s, t)
    ref = oracle.fw_exact(G, 2, 30, with_split=False)
    out = lds.lds_frank_wolfe(g, 2, 30, want_num=True)
    np.testing.assert_array_equal(out["num"], ref["A"])


def disjoint_copies(c, nk=5, L=5):
    """c disjoint copies of K_nk with a cycle through L new vertices and the
    clique's last vertex (cycle vertices have core 2, so pruning keeps them)"""
    s, t, per = [], [], nk + L
    for i in range(c):
        b = i * per
        for a in range(nk):
            for d in range(a + 1, nk):
                s.append(b + a)
                t.append(b + d)
        prev = b + nk - 1
        for j in range(L):
            s.append(prev)
            t.append(b + nk + j)
            prev = b + nk + j
        s.append(prev)
        t.append(b + nk - 1)
    return c * per, np.array(s, np.int32), np.array(t, np.int32)


@pytest.mark.parametrize("iters", [0, 1, 2, 3])
def test_refinements_batched(iters):
    """With 1 or 3 iterations the whole graph of 6 disjoint copies is one
    stable group and no vertex is pruned: its 6 components share the bound,
    each fails IsDensest (16/10 < 2), and their refinements share batched FW
    launches.  Results equal the oracle's for every iteration count."""
    announce("topk batched refinements", iters)
    n, s, t = disjoint_copies(6)
    got, st = check(n, s, t, 2, 6, iters)
    assert len(got) == 6 and all(r == 2 for _, r in got)
    if iters in (1, 3):
        assert st["refinements"] >= 6 and st["refine_rounds"] < st["refinements"]


def test_pruning_running_example():
    """The device pruning (Alg. 3) as lds_topk runs it, on the running example
    with 200 FW iterations: rule 1 removes r, g and i and rule 2 then removes
    o, p, q and h, as in Section 5.2's example."""
    announce("prune running example")
    d, n, s, t = running_example()
    g = lds.lds_create_graph(n, s, t)
    rule, cnt, _ = lds.lds_prune(g, 2, 200)
    assert sorted(np.flatnonzero(rule == 1).tolist()) == sorted(d["pruned_rule1"])
    assert sorted(np.flatnonzero(rule == 2).tolist()) == sorted(d["pruned_rule2"])
    assert cnt == 7


@pytest.mark.parametrize("mode", [2, 3])
def test_pruning_within_exact_pruning(mode):
    """The library's bounds bracket phi, so what it prunes is also pruned by
    Alg. 3 with the exact compact numbers as bounds (the oracle's pruning;
    tighter bounds prune more), and no pruned vertex lies in an LDS."""
    cases = [synth.workload("lds_small")[:3], synth.holme_kim(1500, 5, 0.6, seed=8),
             synth.powerlaw_planted(2500, 2.2, 10.0, n_blocks=8, s_lo=15, s_hi=60, p_block=0.4, seed=9)]
    for n, s, d in cases:
        announce("prune subset", mode, n)
        G = oracle.Graph(n, s, d)
        pn, pd = oracle.decompose(G, mode)
        phi = [Fraction(int(a), int(b)) for a, b in zip(pn, pd)]
        exact = oracle.prune(G, mode, phi, phi)
        g = lds.lds_create_graph(n, s, d)
        for iters in (5, 100):
            rule, cnt, _ = lds.lds_prune(g, mode, iters)
            assert cnt == int((rule != 0).sum())
            assert (exact[rule != 0] != 0).all()
            for vs, _ in oracle.lds_from_phi(G, pn, pd):
                assert (rule[vs] == 0).all()
