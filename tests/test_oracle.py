"""Pins for the CPU oracle: values the paper prints, closed forms, invariants
and brute force, so that the oracle is checked against something other than
itself before any GPU result is compared with it."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def running_example():
    with open(os.path.join(GOLD, "running_example.json")) as f:
        d = json.load(f)
    e = np.array(d["edges"], np.int32)
    return d, oracle.Graph(d["n"], e[:, 0], e[:, 1])


def frac(p):
    return Fraction(p[0], p[1])


def small_graphs():
    """Seeded small graphs of several shapes for brute-force comparison."""
    out = []
    for seed in range(6):
        out.append(synth.erdos_renyi(9 + seed % 4, 0.35 + 0.05 * seed, seed=seed))
    for seed in range(4):
        out.append(synth.powerlaw_planted(12, 2.3, 3.0, 1, 5, 6, 0.9, seed=100 + seed))
    out.append(synth.holme_kim(12, 3, 0.6, seed=7))
    return out


# ---------------------------------------------------------------- running example
def test_running_example_phi_and_lds():
    d, G = running_example()
    assert G.m == 35
    pn, pd = oracle.decompose(G, 2)
    for name, vs in d["groups"].items():
        for u in vs:
            assert Fraction(int(pn[u]), int(pd[u])) == frac(d["phi"][name]), (name, u)
    lds = oracle.lds_from_phi(G, pn, pd)
    assert [(sorted(s.tolist()), r) for s, r in lds] == [(sorted(s), frac(r)) for s, r in d["lds"]]
    # sum of r* equals m (the loads are a feasible split of every edge, Eq. cp)
    assert sum(Fraction(int(a), int(b)) for a, b in zip(pn, pd)) == 35


def test_running_example_triangles_and_ltds():
    d, G = running_example()
    tri, cnt = oracle.triangles(G)
    assert len(tri) == d["num_triangles"] == 32
    assert cnt.sum() == 3 * 32
    pn, pd = oracle.decompose(G, 3)
    for name, vs in d["groups"].items():
        for u in vs:
            assert Fraction(int(pn[u]), int(pd[u])) == frac(d["phi_tr"][name]), (name, u)
    ltds = oracle.lds_from_phi(G, pn, pd)
    assert [(sorted(s.tolist()), r) for s, r in ltds] == [(sorted(s), frac(r)) for s, r in d["ltds"]]


def test_running_example_compactness_examples():
    """S1 u S3: density 21/10, compactness 3/2; tr-density 11/5, tr-compactness
    1/2 (Section 3 and Section 6.1 examples), by enumeration over removal sets."""
    d, G = running_example()
    u, v = G.edges()
    tri, _ = oracle.triangles(G)
    S = set(d["groups"]["S1"]) | set(d["groups"]["S3"])

    def inside(pats, X):
        return sum(1 for p in pats if all(int(x) in X for x in p))

    edges = list(zip(u.tolist(), v.tolist()))
    tris = [tuple(t) for t in tri.tolist()]
    assert Fraction(inside(edges, S), len(S)) == Fraction(21, 10)
    assert Fraction(inside(tris, S), len(S)) == Fraction(11, 5)
    S3 = set(d["groups"]["S3"])
    assert inside(edges, S) - inside(edges, S - S3) == 6
    assert inside(tris, S) - inside(tris, S - S3) == 2
    best_e = best_t = None
    Sl = sorted(S)
    for k in range(1, len(Sl) + 1):
        for Q in itertools.combinations(Sl, k):
            R = S - set(Q)
            fe = Fraction(inside(edges, S) - inside(edges, R), k)
            ft = Fraction(inside(tris, S) - inside(tris, R), k)
            best_e = fe if best_e is None else min(best_e, fe)
            best_t = ft if best_t is None else min(best_t, ft)
    assert best_e == Fraction(3, 2)
    assert best_t == Fraction(1, 2)


def test_running_example_fw_converges_to_phi():
    """Thm. 1: FW's loads approach r* = phi; the error shrinks with N."""
    d, G = running_example()
    phi = np.zeros(G.n)
    for name, vs in d["groups"].items():
        phi[vs] = float(frac(d["phi"][name]))
    errs = []
    for N in (25, 100, 400, 1600):
        out = oracle.fw_exact(G, 2, N, with_gap=False, with_split=False)
        r = out["A"].astype(np.float64) / out["D"]
        errs.append(np.abs(r - phi).max())
    assert errs[-1] < 0.01
    assert errs[0] > errs[-1]


def test_running_example_prefix_at_phi():
    """Alg. 2's sort and prefix densities at r* (loads proportional to phi, ties by id):
    hand-derived E_j and I = {6, 11, 12, 15, 16, 18} (1-based)."""
    d, G = running_example()
    L = 12  # common multiple of all phi denominators
    A = np.zeros(G.n, np.uint64)
    for name, vs in d["groups"].items():
        A[vs] = int(frac(d["phi"][name]) * L)
    order, E, inI = oracle.sort_prefix(G, 2, A)
    assert order.tolist() == [0, 1, 2, 3, 4, 5, 9, 10, 11, 12, 13, 14, 15, 16, 17, 6, 7, 8]
    assert E.tolist() == [0, 1, 3, 6, 10, 15, 15, 16, 18, 21, 25, 25, 26, 27, 31, 32, 33, 35]
    assert (np.flatnonzero(inI) + 1).tolist() == [6, 11, 12, 15, 16, 18]


def test_running_example_extract_sg_after_convergence():
    """At a well-converged FW iterate the stable groups are S1, S2, S3, S4
    (Section 5.1, Fig. stable groups) and their bounds bracket phi
    (Lemma phi-bounds)."""
    d, G = running_example()
    N = 2000
    out = oracle.fw_exact(G, 2, N, with_gap=False)
    groups, lo, hi = oracle.extract_sg(G, 2, out["A"], out["split"], out["D"])
    order, _, _ = oracle.sort_prefix(G, 2, out["A"])
    sets = [sorted(order[s:e].tolist()) for s, e in groups]
    assert sets == [sorted(d["groups"][k]) for k in ("S1", "S2", "S3", "S4")]
    for name, vs in d["groups"].items():
        for u in vs:
            ph = frac(d["phi"][name])
            assert Fraction(int(lo[u]), out["D"]) <= ph <= Fraction(int(hi[u]), out["D"])


# ------------------------------------------------------------------ closed forms
def test_star_first_iterations():
    """Star K_{1,d}: r0 = (d/2, 1/2...), after one FW step every leaf wins its
    edge: hub d/6, leaves 5/6; phi = d/(d+1) everywhere."""
    d = 7
    G = oracle.Graph(d + 1, np.zeros(d, np.int32), np.arange(1, d + 1, dtype=np.int32))
    out = oracle.fw_exact(G, 2, 1)
    assert out["D"] == 6
    assert out["A"].tolist() == [d] + [5] * d
    pn, pd = oracle.decompose(G, 2)
    assert all(Fraction(int(a), int(b)) == Fraction(d, d + 1) for a, b in zip(pn, pd))


def test_k3_hand_iterations():
    """K_3 with ties broken towards the larger id (Alg. 1's else branch):
    A^1=(2,6,10)/6, A^2=(14,12,10)/12, A^3=(14,20,26)/20."""
    G = oracle.Graph(3, np.array([0, 0, 1], np.int32), np.array([1, 2, 2], np.int32))
    for N, want, D in ((1, [2, 6, 10], 6), (2, [14, 12, 10], 12), (3, [14, 20, 26], 20)):
        out = oracle.fw_exact(G, 2, N)
        assert out["D"] == D
        assert out["A"].tolist() == want


def test_kn_phi():
    for n in (4, 6, 9):
        u, v = zip(*itertools.combinations(range(n), 2))
        G = oracle.Graph(n, np.array(u, np.int32), np.array(v, np.int32))
        pn, pd = oracle.decompose(G, 2)
        assert all(Fraction(int(a), int(b)) == Fraction(n - 1, 2) for a, b in zip(pn, pd))
        pn, pd = oracle.decompose(G, 3)
        assert all(Fraction(int(a), int(b)) == Fraction((n - 1) * (n - 2), 6) for a, b in zip(pn, pd))
        tri, cnt = oracle.triangles(G)
        assert len(tri) == n * (n - 1) * (n - 2) // 6


def test_triangle_first_iteration_single_triangle():
    """One triangle: r0 = 1/3 each (alpha = 1/3, Alg. 6 init); iteration 1
    gives the unit to the largest id: A=(2,2,2+12)/18 -> (1/9,1/9,7/9)."""
    G = oracle.Graph(3, np.array([0, 0, 1], np.int32), np.array([1, 2, 2], np.int32))
    out = oracle.fw_exact(G, 3, 1)
    assert out["D"] == 18
    assert out["A"].tolist() == [2, 2, 14]
    assert out["split"].tolist() == [[2, 2, 14]]


# ------------------------------------------------------------------- brute force
@pytest.mark.parametrize("mode", [2, 3])
def test_decomposition_matches_brute_force(mode):
    for n, s, d in small_graphs():
        G = oracle.Graph(n, s, d)
        phi_b, sets_b = oracle.brute(G, mode)
        pn, pd = oracle.decompose(G, mode)
        phi_d = [Fraction(int(a), int(b)) for a, b in zip(pn, pd)]
        assert phi_d == phi_b
        sets_d = oracle.lds_from_phi(G, pn, pd)
        assert [(s.tolist(), r) for s, r in sets_d] == [(s.tolist(), r) for s, r in sets_b]


def test_triangles_brute_force():
    for n, s, d in small_graphs() + [synth.powerlaw_planted(60, 2.3, 6.0, 2, 6, 10, 0.7, seed=9)]:
        G = oracle.Graph(n, s, d)
        u, v = G.edges()
        E = set(zip(u.tolist(), v.tolist()))
        want = [t for t in itertools.combinations(range(G.n), 3)
                if (t[0], t[1]) in E and (t[0], t[2]) in E and (t[1], t[2]) in E]
        tri, cnt = oracle.triangles(G)
        assert [tuple(t) for t in tri.tolist()] == want
        c = np.zeros(G.n, np.int64)
        for t in want:
            for x in t:
                c[x] += 1
        assert cnt.tolist() == c.tolist()


# ---------------------------------------------------------------- FW invariants
@pytest.mark.parametrize("mode", [2, 3])
def test_fw_invariants_and_gap(mode):
    n, s, d = synth.powerlaw_planted(300, 2.3, 8.0, 3, 10, 20, 0.5, seed=11)
    G = oracle.Graph(n, s, d)
    N = 60
    out = oracle.fw_exact(G, mode, N)
    D = out["D"]
    P = out["split"].shape[0]
    # Eq. cp / trcp constraints: every pattern's split sums to one
    assert (out["split"].sum(axis=1) == D).all()
    assert (out["split"] >= 0).all()
    assert int(out["A"].sum()) == D * P
    # loads are the sum of the splits (r_u = sum alpha)
    pats = np.stack(G.edges(), 1) if mode == 2 else oracle.triangles(G)[0]
    r = np.zeros(G.n, np.int64)
    np.add.at(r, pats.reshape(-1), out["split"].astype(np.int64).reshape(-1))
    assert (r == out["A"].astype(np.int64)).all()
    # duality gap: g >= 0 and g >= f - f* (f* = sum phi^2, Thm. 1 / Thm. cp)
    pn, pd = oracle.decompose(G, mode)
    fstar = float(sum(Fraction(int(a), int(b)) ** 2 for a, b in zip(pn, pd)))
    gap, lb = out["gap"], out["lb"]
    assert (gap >= -1e-9).all()
    assert (lb <= fstar * (1 + 1e-12) + 1e-9).all()
    # certified gap min f - max lb is non-increasing and >= 0
    f = gap + lb
    cert = np.minimum.accumulate(f) - np.maximum.accumulate(lb)
    assert (np.diff(cert) <= 1e-9).all() and (cert >= -1e-9).all()


@pytest.mark.parametrize("mode", [2, 3])
def test_fw_exact_matches_literal_fp64(mode):
    """The exact-rational iteration and the FP64 transcription of Alg. 1 / 6
    agree after the first step (r0 = deg/2 or t/3 ties are resolved the same
    way), and both approach phi.  In between they drift apart: FP64 rounding
    breaks exact ties differently, which is why decisions are taken on exact
    numerators."""
    n, s, d = synth.powerlaw_planted(200, 2.3, 6.0, 2, 8, 12, 0.6, seed=21)
    G = oracle.Graph(n, s, d)
    ex = oracle.fw_exact(G, mode, 1)
    r_lit, al_lit = oracle.fw_literal(G, mode, 1)
    r_ex = ex["A"].astype(np.float64) / ex["D"]
    assert np.abs(r_ex - r_lit).max() < 1e-12
    assert np.abs(ex["split"].astype(np.float64) / ex["D"] - al_lit).max() < 1e-15
    pn, pd = oracle.decompose(G, mode)
    phi = pn / pd
    N = 2000
    r_lit, _ = oracle.fw_literal(G, mode, N)
    ex = oracle.fw_exact(G, mode, N, with_gap=False, with_split=False)
    r_ex = ex["A"].astype(np.float64) / ex["D"]
    assert np.abs(r_lit - phi).max() < 0.05
    assert np.abs(r_ex - phi).max() < 0.05


def test_fw_converges_on_random_graphs():
    for n, s, d in small_graphs()[:6]:
        G = oracle.Graph(n, s, d)
        pn, pd = oracle.decompose(G, 2)
        phi = pn / pd
        out = oracle.fw_exact(G, 2, 3000, with_gap=False, with_split=False)
        r = out["A"].astype(np.float64) / out["D"]
        assert np.abs(r - phi).max() < 0.02


# ---------------------------------------------------------- ExtractSG properties
@pytest.mark.parametrize("mode", [2, 3])
def test_extract_sg_bounds_and_stability(mode):
    """Lemma phi-bounds / tr-phi-bounds against exact phi, and Def. 5 condition
    1 on the restricted loads, on a planted power-law graph."""
    n, s, d = synth.powerlaw_planted(400, 2.3, 6.0, 4, 10, 25, 0.5, seed=31)
    G = oracle.Graph(n, s, d)
    N = 150
    out = oracle.fw_exact(G, mode, N)
    D = out["D"]
    groups, lo, hi = oracle.extract_sg(G, mode, out["A"], out["split"], D)
    assert len(groups) > 0
    order, E, inI = oracle.sort_prefix(G, mode, out["A"])
    ends = set((np.flatnonzero(inI) + 1).tolist())
    pn, pd = oracle.decompose(G, mode)
    prev_lo = None
    for (a, b) in groups:
        assert b in ends  # groups are unions of consecutive candidates
        vs = order[a:b]
        assert len(set(lo[vs].tolist())) == 1 and len(set(hi[vs].tolist())) == 1
        glo, ghi = int(lo[vs[0]]), int(hi[vs[0]])
        assert glo <= ghi
        if prev_lo is not None:
            assert ghi < prev_lo  # strictly below the group above (condition 1)
        prev_lo = glo
        for u in vs:
            ph = Fraction(int(pn[u]), int(pd[u]))
            assert Fraction(glo, D) <= ph <= Fraction(ghi, D), (u, glo, ghi, ph)
    # consecutive groups tile a prefix of the order
    assert groups[0][0] == 0
    for (a, b), (c, e) in zip(groups, groups[1:]):
        assert b == c


def test_prefix_invariants():
    n, s, d = synth.powerlaw_planted(500, 2.3, 8.0, 3, 10, 30, 0.5, seed=41)
    G = oracle.Graph(n, s, d)
    out = oracle.fw_exact(G, 2, 50, with_gap=False, with_split=False)
    order, E, inI = oracle.sort_prefix(G, 2, out["A"])
    assert sorted(order.tolist()) == list(range(G.n))
    A = out["A"][order]
    assert (A[:-1] >= A[1:]).all()
    assert (np.diff(E) >= 0).all() and E[-1] == G.m
    assert inI[-1]
    # brute force suffix argmax with ties to the larger index
    dens = [Fraction(int(E[j]), j + 1) for j in range(G.n)]
    for i in range(0, G.n, 37):
        best = max(range(i, G.n), key=lambda j: (dens[j], j))
        assert inI[best]


# ---------------------------------------------------------------- core numbers
def _core_by_enumeration(n, edges, mode):
    """core(u) = max over vertex sets X containing u of the smallest number of
    patterns inside X at a vertex of X (every subset enumerated)."""
    import itertools
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    best = [0] * n
    for mask in range(1, 1 << n):
        X = [u for u in range(n) if (mask >> u) & 1]
        inX = set(X)
        if mode == 2:
            cnt = {u: len(adj[u] & inX) for u in X}
        else:
            cnt = {u: 0 for u in X}
            for a, b, c in itertools.combinations(X, 3):
                if b in adj[a] and c in adj[a] and c in adj[b]:
                    cnt[a] += 1
                    cnt[b] += 1
                    cnt[c] += 1
        m = min(cnt.values())
        for u in X:
            best[u] = max(best[u], m)
    return best


def test_core_numbers_closed_forms():
    # K_n: every vertex has core n-1 and tr-core C(n-1, 2)
    for n in (3, 5, 8):
        s, d = np.triu_indices(n, 1)
        G = oracle.Graph(n, s.astype(np.int32), d.astype(np.int32))
        assert (oracle.core_numbers(G, 2) == n - 1).all()
        assert (oracle.core_numbers(G, 3) == (n - 1) * (n - 2) // 2).all()
    # star: core 1 everywhere, no triangles; cycle: core 2
    G = oracle.Graph(6, np.zeros(5, np.int32), np.arange(1, 6, dtype=np.int32))
    assert list(oracle.core_numbers(G, 2)) == [1] * 6
    assert list(oracle.core_numbers(G, 3)) == [0] * 6
    G = oracle.Graph(7, np.arange(7, dtype=np.int32), ((np.arange(7) + 1) % 7).astype(np.int32))
    assert list(oracle.core_numbers(G, 2)) == [2] * 7
    # an isolated vertex keeps 0
    G = oracle.Graph(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    assert list(oracle.core_numbers(G, 2)) == [1, 1, 1, 0]


def test_core_numbers_by_enumeration():
    rng = np.random.default_rng(3)
    for trial in range(12):
        n = int(rng.integers(4, 11))
        edges = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < 0.45]
        if not edges:
            continue
        e = np.array(edges, np.int32)
        G = oracle.Graph(n, e[:, 0].copy(), e[:, 1].copy())
        for mode in (2, 3):
            assert list(oracle.core_numbers(G, mode)) == _core_by_enumeration(n, edges, mode)


# ------------------------------------------------------------- pruning
def test_pruning_running_example():
    """Alg. 3 on the running example with the exact compact numbers as both
    bounds: rule 1 removes r, g and i, rule 2 then removes o, p, q and h
    (Section 5.2's example)."""
    d, G = running_example()
    pn, pd = oracle.decompose(G, 2)
    phi = [Fraction(int(a), int(b)) for a, b in zip(pn, pd)]
    rule = oracle.prune(G, 2, phi, phi)
    assert sorted(np.flatnonzero(rule == 1).tolist()) == sorted(d["pruned_rule1"])
    assert sorted(np.flatnonzero(rule == 2).tolist()) == sorted(d["pruned_rule2"])


@pytest.mark.parametrize("mode", [2, 3])
def test_pruning_keeps_every_lds(mode):
    """No vertex of an LDS (LTDS) is removed by Alg. 3 with exact bounds (the
    rules' claim), on random small graphs against brute force."""
    for n, s, d in small_graphs():
        G = oracle.Graph(n, s, d)
        phi, sets = oracle.brute(G, mode)
        rule = oracle.prune(G, mode, phi, phi)
        for vs, _ in sets:
            assert (rule[vs] == 0).all()


# ------------------------------------------ large-graph path (k-core, superlevel)
def _helper_graphs():
    return small_graphs() + [synth.powerlaw_planted(300, 2.3, 6.0, 3, 8, 20, 0.6, seed=9),
                             synth.holme_kim(300, 4, 0.6, seed=9)]


def test_kcore_matches_core_numbers():
    """One k-core by deletion equals {core >= k} of the core numbers above
    (pinned by enumeration), for every k from 0 to one past the largest."""
    for n, s, d in _helper_graphs():
        G = oracle.Graph(n, s, d)
        for mode in (2, 3):
            core = oracle.core_numbers(G, mode)
            for k in range(int(core.max()) + 2):
                np.testing.assert_array_equal(oracle.kcore(G, mode, k), core >= k)


def test_superlevel_matches_decomposition():
    """{phi >= lam} by one min cut equals the union of the decomposition's
    levels of density >= lam (pinned against brute force above): at every
    level value (the tie case: the level itself belongs), between levels,
    at 0 and above the top."""
    for n, s, d in _helper_graphs():
        G = oracle.Graph(n, s, d)
        for mode in (2, 3):
            pn, pd = oracle.decompose(G, mode)
            phi = [Fraction(int(a), int(b)) for a, b in zip(pn, pd)]
            lv = sorted(set(phi))
            lams = set(lv) | {(a + b) / 2 for a, b in zip(lv, lv[1:])} | {lv[-1] + Fraction(1, 3), Fraction(0)}
            for lam in sorted(lams):
                want = np.array([f >= lam for f in phi])
                np.testing.assert_array_equal(oracle.superlevel(G, mode, lam), want)


@pytest.mark.parametrize("mode", [2, 3])
def test_top_levels_matches_full_top_k(mode):
    """The large-graph path (k-core, one superlevel min cut, decomposition of
    the superlevel set only) returns exactly the sets of the full
    decomposition's LDS / LTDS list with density >= lam, in the same order."""
    graphs = [synth.workload("lds_small")[:3], synth.powerlaw_planted(1500, 2.1, 10.0, 6, 15, 60, 0.4, seed=21),
              synth.holme_kim(1200, 6, 0.6, seed=22)]
    for n, s, d in graphs:
        G = oracle.Graph(n, s, d)
        full = oracle.lds_from_phi(G, *oracle.decompose(G, mode))
        dens = sorted({r for _, r in full}, reverse=True)
        lams = {dens[0], dens[-1], dens[min(2, len(dens) - 1)], dens[0] / 2}
        if len(dens) > 1:
            lams.add((dens[0] + dens[1]) / 2)
        for lam in sorted(lams):
            got, K, U = oracle.top_levels(G, mode, lam)
            want = [(v, r) for v, r in full if r >= lam]
            assert len(got) == len(want) and U <= K <= n
            for (gv, gr), (wv, wr) in zip(got, want):
                assert gr == wr
                np.testing.assert_array_equal(gv, wv)


# ------------------------------------------------------- 4-clique program (h = 4)
def clique_graphs():
    """small graphs with 4-cliques: dense G(n,p), planted blocks, triadic closure"""
    out = [synth.erdos_renyi(10 + s % 3, 0.55 + 0.05 * s, seed=40 + s) for s in range(4)]
    out += [synth.powerlaw_planted(12, 2.3, 3.0, 2, 5, 6, 0.95, seed=50 + s) for s in range(3)]
    out.append(synth.holme_kim(12, 4, 0.8, seed=8))
    return out


def test_cliques4_by_enumeration():
    for n, s, d in clique_graphs() + [synth.powerlaw_planted(60, 2.3, 6.0, 2, 8, 12, 0.8, seed=9)]:
        G = oracle.Graph(n, s, d)
        u, v = G.edges()
        E = set(zip(u.tolist(), v.tolist()))
        want = [q for q in itertools.combinations(range(G.n), 4)
                if all((q[i], q[j]) in E for i in range(4) for j in range(i + 1, 4))]
        got, cnt = oracle.cliques4(G)
        assert [tuple(x) for x in got.tolist()] == want
        c = np.zeros(G.n, np.int64)
        for q in want:
            c[list(q)] += 1
        assert cnt.tolist() == c.tolist()
    assert sum(len(oracle.cliques4(oracle.Graph(*g))[0]) for g in clique_graphs()) > 20


def test_fw4_hand_iterations_k4_k5():
    """K4: r0 = 1/4 each (D0 = 4, numerators 1).  Iteration 1: all tie, the
    largest id wins, inc = 4*2: A = (1,1,1,9) / 12.  Iteration 2: ids 0..2 tie
    at 1, id 2 wins, inc 12: (1,1,13,9) / 24.  Iteration 3: ids 0, 1 tie, id 1
    wins, inc 16: (1,17,13,9) / 40.  K5: every vertex lies in 4 of the 5
    4-cliques, r0 = 1 (A = 4 over D0 = 4)."""
    k4 = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    G = oracle.Graph(4, np.array([e[0] for e in k4], np.int32), np.array([e[1] for e in k4], np.int32))
    want = {0: ([1, 1, 1, 1], 4), 1: ([1, 1, 1, 9], 12), 2: ([1, 1, 13, 9], 24), 3: ([1, 17, 13, 9], 40)}
    for it, (A, D) in want.items():
        out = oracle.fw_exact(G, 4, it)
        assert out["A"].tolist() == A and out["D"] == D
        assert out["split"].tolist() == [A]  # one clique: its split is the load
    # the uniform start is optimal on K4: zero gap at r0
    assert oracle.fw_exact(G, 4, 1)["gap"][0] == 0.0
    k5 = [(a, b) for a in range(5) for b in range(a + 1, 5)]
    G = oracle.Graph(5, np.array([e[0] for e in k5], np.int32), np.array([e[1] for e in k5], np.int32))
    assert oracle.fw_exact(G, 4, 0)["A"].tolist() == [4] * 5
    # no 4-clique: nothing to route
    tri = oracle.Graph(3, np.array([0, 1, 0], np.int32), np.array([1, 2, 2], np.int32))
    out = oracle.fw_exact(tri, 4, 5)
    assert out["A"].tolist() == [0, 0, 0] and out["split"].shape == (0, 4)


def test_fw4_invariants():
    n, s, d = synth.powerlaw_planted(200, 2.3, 6.0, 3, 8, 14, 0.7, seed=31)
    G = oracle.Graph(n, s, d)
    q, cnt = oracle.cliques4(G)
    assert len(q) > 100
    out = oracle.fw_exact(G, 4, 50)
    D = out["D"]
    assert D == 2 * 51 * 52
    assert (out["split"].sum(axis=1) == D).all() and (out["split"] >= 0).all()
    assert int(out["A"].sum()) == D * len(q)
    r = np.zeros(G.n, np.int64)
    np.add.at(r, q.reshape(-1), out["split"].astype(np.int64).reshape(-1))
    assert (r == out["A"].astype(np.int64)).all()
    assert (out["gap"] >= 0).all()
    # the first iterate is the initial quarter shares
    assert (oracle.fw_exact(G, 4, 0)["A"] == cnt).all()
    # the FP64 transcription takes the same first step
    r_lit, al_lit = oracle.fw_literal(G, 4, 1)
    ex = oracle.fw_exact(G, 4, 1)
    assert np.abs(ex["A"] / ex["D"] - r_lit).max() < 1e-12
    assert np.abs(ex["split"] / ex["D"] - al_lit).max() < 1e-15


def clique_levels(n, cliques):
    """Optimum of the 4-clique program by brute force over vertex subsets: the
    nested sets B_1 < B_2 < ... of the density-friendly decomposition, each the
    largest U above B_{i-1} maximising (c(U) - c(B_{i-1})) / (|U| - |B_{i-1}|),
    c(U) = 4-cliques inside U; every vertex of B_i \\ B_{i-1} gets that ratio."""
    masks = [sum(1 << x for x in q) for q in cliques]
    c = [sum(1 for m in masks if (U & m) == m) for U in range(1 << n)]
    r = [Fraction(0)] * n
    B = 0
    while B != (1 << n) - 1:
        best, top = None, 0
        for U in range(1 << n):
            if U & B != B or U == B:
                continue
            lam = Fraction(c[U] - c[B], bin(U).count("1") - bin(B).count("1"))
            if best is None or lam > best:
                best, top = lam, U
            elif lam == best:
                top |= U
        for x in range(n):
            if (top >> x) & 1 and not (B >> x) & 1:
                r[x] = best
        B = top
    return r


def test_fw4_converges_to_the_brute_force_optimum():
    """||r - r*||^2 <= f(r) - f(r*) <= gap(r) for f = sum r^2 (strong convexity
    and the Frank-Wolfe duality gap), with r* from the decomposition above and
    the gap computed from its definition 2 (sum r^2 - sum_q min_{x in q} r_x)."""
    for n, s, d in clique_graphs():
        G = oracle.Graph(n, s, d)
        q, _ = oracle.cliques4(G)
        rstar = np.array([float(x) for x in clique_levels(G.n, q.tolist())])
        out = oracle.fw_exact(G, 4, 1500, with_gap=False, with_split=False)
        r = out["A"].astype(np.float64) / out["D"]
        gap = 2.0 * (np.sum(r * r) - (r[q].min(axis=1).sum() if len(q) else 0.0))
        assert gap >= -1e-12
        assert np.sum((r - rstar) ** 2) <= gap + 1e-12
        assert np.abs(r - rstar).max() < 0.1
        # the densest 4-clique density is the largest level
        assert abs(r.max() - rstar.max()) < 0.1
