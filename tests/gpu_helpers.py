"""Shared helpers of the GPU parity tests: run the same seeded input through
the library (C ABI via the binding) and through the oracle, and compare."""
import sys

import numpy as np

import oracle
import paper_2504_10937_amd as lds


def announce(*what):
    print("[case]", *what, flush=True)
    sys.stdout.flush()


def edge_split_map(G):
    """oracle: {(u,v) canonical: (a_u, a_v)} from fw_exact splits"""
    u, v = G.edges()
    return u, v


def lex_lower_bound(rows, keys):
    """first index i with rows[i] >= key (lexicographic), for every key row;
    rows sorted lexicographically (vectorised binary search)"""
    N = len(rows)
    lo = np.zeros(len(keys), np.int64)
    hi = np.full(len(keys), N, np.int64)
    while True:
        active = lo < hi
        if not active.any():
            return lo
        mid = (lo + hi) // 2
        r = rows[np.minimum(mid, N - 1)]
        less = np.zeros(len(keys), bool)
        eq = np.ones(len(keys), bool)
        for c in range(rows.shape[1]):
            less |= eq & (r[:, c] < keys[:, c])
            eq &= r[:, c] == keys[:, c]
        lo = np.where(active & less, mid + 1, lo)
        hi = np.where(active & ~less, mid, hi)


def check_fw(n, src, dst, mode, iters, gap=True, G=None, gpu_graph=None):
    """Run FW on both sides; assert exact numerators, splits and gap."""
    if G is None:
        G = oracle.Graph(n, src, dst)
    g = gpu_graph if gpu_graph is not None else lds.lds_create_graph(n, src, dst)
    out = lds.lds_frank_wolfe(g, mode, iters, want_r64=True, want_num=True, want_gap=gap)
    ref = oracle.fw_exact(G, mode, iters, with_gap=gap)
    assert out["D"] == ref["D"]
    np.testing.assert_array_equal(out["num"], ref["A"])
    np.testing.assert_array_equal(out["r64"], ref["A"].astype(np.float64) / ref["D"])
    if gap and iters > 0:
        np.testing.assert_allclose(out["gap"], ref["gap"], rtol=1e-12, atol=1e-12 * max(1.0, float(np.abs(ref["gap"]).max())))
    # splits: every incidence (x, pattern) numerator equals the oracle's
    verts, num = lds.lds_splits(g, mode)
    if mode == 2:
        u, v = G.edges()
        assert len(num) == 2 * G.m
        key_o = u.astype(np.int64) * n + v
        order = np.argsort(key_o)
        x, y = verts[:, 0].astype(np.int64), verts[:, 1].astype(np.int64)
        key = np.minimum(x, y) * n + np.maximum(x, y)
        idx = order[np.searchsorted(key_o[order], key)]
        assert (key_o[idx] == key).all()
        want = np.where(x < y, ref["split"][idx, 0], ref["split"][idx, 1])
        np.testing.assert_array_equal(num, want)
    else:
        pats = oracle.triangles(G)[0] if mode == 3 else oracle.cliques4(G)[0]
        assert len(num) == mode * len(pats)
        if len(pats):
            # patterns are sorted ascending tuples: match them by their sorted rows
            p64 = pats.astype(np.int64)
            s = np.sort(verts.astype(np.int64), axis=1)
            order = np.lexsort(p64.T[::-1])
            assert (order == np.arange(len(p64))).all()  # the oracle's list is lexicographic
            idx = lex_lower_bound(p64, s)
            assert (idx < len(p64)).all() and (p64[idx] == s).all()
            pos = np.argmax(p64[idx] == verts[:, :1].astype(np.int64), axis=1)
            want = ref["split"][idx, pos]
            np.testing.assert_array_equal(num, want)
    return g, G, out, ref
