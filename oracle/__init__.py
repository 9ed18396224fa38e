"""Python binding of the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
module and this module never imports the GPU library; the two share only the
seeded input generators of the ``synth`` package.

Every function is a thin ctypes marshalling layer over the C code, which
follows the paper (arXiv 2504.10937) section by section; see ``oracle.c``.
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile the oracle in-tree with gcc."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", os.path.join(_HERE, "oracle.c"),
                           "-o", tmp, "-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    L = ctypes.CDLL(_SO)
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    sig = {
        "orc_graph_new": (vp, [i64, i64, vp, vp]),
        "orc_graph_free": (None, [vp]),
        "orc_graph_n": (i64, [vp]),
        "orc_graph_m": (i64, [vp]),
        "orc_graph_edges": (None, [vp, vp, vp]),
        "orc_graph_degrees": (None, [vp, vp]),
        "orc_triangles": (i64, [vp, vp, vp]),
        "orc_cliques4": (i64, [vp, vp, vp]),
        "orc_fw_exact": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]),
        "orc_fw_literal": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp]),
        "orc_sort_prefix": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp, vp]),
        "orc_extract_sg": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, u64, vp, vp, vp, vp, vp]),
        "orc_decompose": (i64, [vp, ctypes.c_int, vp, vp]),
        "orc_core_numbers": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "orc_lds_from_phi": (i64, [vp, vp, vp, vp, vp, vp, vp]),
        "orc_brute": (i64, [vp, ctypes.c_int, vp, vp, vp, vp, vp]),
        "orc_kcore": (i64, [vp, ctypes.c_int, i64, vp]),
        "orc_superlevel": (i64, [vp, ctypes.c_int, i64, i64, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _p(a):
    return a.ctypes.data if a is not None else None


def denominator(mode, iters):
    """Common denominator of the loads after `iters` iterations with
    gamma_i = 2/(i+2): (i+1)(i+2) for edges, 3(i+1)(i+2) for triangles,
    2(i+1)(i+2) for 4-cliques (mode 4)."""
    return {2: 1, 3: 3, 4: 2}[mode] * (iters + 1) * (iters + 2)


class Graph:
    """Simple undirected graph (self-loops dropped, duplicates merged)."""

    def __init__(self, n, src, dst):
        L = _load()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        self._h = L.orc_graph_new(int(n), len(src), _p(src), _p(dst))
        if not self._h:
            raise ValueError("oracle: invalid graph input")
        self.n = int(L.orc_graph_n(self._h))
        self.m = int(L.orc_graph_m(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_graph_free(self._h)
            self._h = None

    def edges(self):
        u = np.empty(self.m, np.int32)
        v = np.empty(self.m, np.int32)
        _load().orc_graph_edges(self._h, _p(u), _p(v))
        return u, v

    def degrees(self):
        d = np.empty(self.n, np.int64)
        _load().orc_graph_degrees(self._h, _p(d))
        return d


def triangles(G):
    """All triangles as a sorted (T,3) array of ascending triples, plus the
    per-vertex triangle counts t_u."""
    L = _load()
    T = L.orc_triangles(G._h, None, None)
    if T < 0:
        raise MemoryError
    tri = np.empty((T, 3), np.int32)
    cnt = np.empty(G.n, np.int64)
    L.orc_triangles(G._h, _p(tri), _p(cnt))
    return tri, cnt


def cliques4(G):
    """All 4-cliques as a sorted (Q,4) array of ascending quadruples, plus the
    per-vertex 4-clique counts."""
    L = _load()
    Q = L.orc_cliques4(G._h, None, None)
    if Q < 0:
        raise MemoryError
    q = np.empty((Q, 4), np.int32)
    cnt = np.empty(G.n, np.int64)
    L.orc_cliques4(G._h, _p(q), _p(cnt))
    return q, cnt


def num_patterns(G, mode):
    if mode == 2:
        return G.m
    if mode == 3:
        return int(_load().orc_triangles(G._h, None, None))
    return int(_load().orc_cliques4(G._h, None, None))


def fw_exact(G, mode, iters, with_gap=True, with_split=True):
    """Alg. 1 (mode 2) / Alg. 6 (mode 3) / the same iteration over 4-cliques
    (mode 4) in exact rational form.

    Returns dict(A=numerators (n,), D=denominator, split=(P,h) numerators in
    canonical pattern order, gap=(iters,), lb=(iters,))."""
    L = _load()
    A = np.empty(G.n, np.uint64)
    P = num_patterns(G, mode) if with_split else 0
    split = np.empty((P, mode), np.uint64) if with_split else None
    gap = np.empty(iters, np.float64) if with_gap else None
    lb = np.empty(iters, np.float64) if with_gap else None
    if L.orc_fw_exact(G._h, mode, iters, _p(A), _p(split), _p(gap), _p(lb)):
        raise RuntimeError("oracle fw_exact failed")
    return {"A": A, "D": denominator(mode, iters), "split": split, "gap": gap, "lb": lb}


def fw_literal(G, mode, iters):
    """Alg. 1 / Alg. 6 as printed, in FP64 -> (r (n,), alpha (P,h))."""
    L = _load()
    P = num_patterns(G, mode)
    r = np.empty(G.n, np.float64)
    al = np.empty((P, mode), np.float64)
    if L.orc_fw_literal(G._h, mode, iters, _p(r), _p(al)):
        raise RuntimeError("oracle fw_literal failed")
    return r, al


def sort_prefix(G, mode, A):
    """Alg. 2, sort by r and prefix densities -> (order, E, inI) (0-based positions)."""
    L = _load()
    A = np.ascontiguousarray(A, dtype=np.uint64)
    order = np.empty(G.n, np.int32)
    E = np.empty(G.n, np.int64)
    inI = np.empty(G.n, np.uint8)
    if L.orc_sort_prefix(G._h, mode, _p(A), _p(order), _p(E), _p(inI)):
        raise RuntimeError("oracle sort_prefix failed")
    return order, E, inI.astype(bool)


def extract_sg(G, mode, A, split, D):
    """Alg. 2 -> (groups [(start,end)], lo (n,), hi (n,)); lo/hi are numerators
    over D, -1 for vertices without bounds."""
    L = _load()
    A = np.ascontiguousarray(A, dtype=np.uint64)
    split = np.ascontiguousarray(split, dtype=np.uint64)
    ng = ctypes.c_int64(0)
    gs = np.empty(max(G.n, 1), np.int64)
    ge = np.empty(max(G.n, 1), np.int64)
    lo = np.empty(G.n, np.int64)
    hi = np.empty(G.n, np.int64)
    if L.orc_extract_sg(G._h, mode, _p(A), _p(split), int(D), ctypes.addressof(ng), _p(gs), _p(ge), _p(lo),
                        _p(hi)):
        raise RuntimeError("oracle extract_sg failed")
    k = ng.value
    return [(int(gs[i]), int(ge[i])) for i in range(k)], lo, hi


def core_numbers(G, mode):
    """Core numbers (mode 2) / tr-core numbers (mode 3) by the definition
    (nested k-cores, repeated deletion) -> int64 array."""
    out = np.empty(G.n, np.int64)
    if _load().orc_core_numbers(G._h, mode, _p(out)) < 0:
        raise RuntimeError("oracle core numbers failed")
    return out


def decompose(G, mode):
    """Exact compact numbers (edges: Def. 4; triangles: Def. trcn) as a list of
    Fractions, via the nested level sets of Thm. 1 / Thm. cp."""
    L = _load()
    pn = np.empty(G.n, np.int64)
    pd = np.empty(G.n, np.int64)
    if L.orc_decompose(G._h, mode, _p(pn), _p(pd)) < 0:
        raise RuntimeError("oracle decompose failed")
    return pn, pd


def lds_from_phi(G, pn, pd):
    """LDS / LTDS sets from exact compact numbers -> list of (sorted vertex
    array, Fraction density), ordered by (density desc, min vertex asc)."""
    L = _load()
    pn = np.ascontiguousarray(pn, dtype=np.int64)
    pd = np.ascontiguousarray(pd, dtype=np.int64)
    comp = np.empty(G.n, np.int64)
    rn = np.empty(max(G.n, 1), np.int64)
    rd = np.empty(max(G.n, 1), np.int64)
    mv = np.empty(max(G.n, 1), np.int64)
    k = L.orc_lds_from_phi(G._h, _p(pn), _p(pd), _p(comp), _p(rn), _p(rd), _p(mv))
    if k < 0:
        raise RuntimeError("oracle lds_from_phi failed")
    out = []
    for i in range(k):
        out.append((np.flatnonzero(comp == i).astype(np.int32), Fraction(int(rn[i]), int(rd[i]))))
    return out


def top_k(G, mode, k):
    """Top-k LDS (mode 2) / LTDS (mode 3) by the definitions (exact)."""
    pn, pd = decompose(G, mode)
    return lds_from_phi(G, pn, pd)[:k]


def brute(G, mode):
    """Enumeration over all subsets (n <= 16) -> (phi as Fractions,
    [(vertex array, Fraction density)] of LDS/LTDS with density > 0)."""
    L = _load()
    if G.n > 16:
        raise ValueError("brute force needs n <= 16")
    pn = np.empty(G.n, np.int64)
    pd = np.empty(G.n, np.int64)
    cap = 1 << G.n
    masks = np.empty(max(cap, 1), np.uint32)
    ln = np.empty(max(cap, 1), np.int64)
    ld = np.empty(max(cap, 1), np.int64)
    k = L.orc_brute(G._h, mode, _p(pn), _p(pd), _p(masks), _p(ln), _p(ld))
    if k < 0:
        raise RuntimeError("oracle brute failed")
    phi = [Fraction(int(a), int(b)) for a, b in zip(pn, pd)]
    sets = []
    for i in range(k):
        vs = np.array([u for u in range(G.n) if (int(masks[i]) >> u) & 1], np.int32)
        sets.append((vs, Fraction(int(ln[i]), int(ld[i]))))
    return phi, sets


def kcore(G, mode, k):
    """The k-core (mode 2) / k-tr-core (mode 3) by repeated deletion -> bool (n,)."""
    m = np.empty(G.n, np.uint8)
    if _load().orc_kcore(G._h, mode, int(k), _p(m)) < 0:
        raise RuntimeError("oracle kcore failed")
    return m.astype(bool)


def superlevel(G, mode, lam):
    """{u : phi(u) >= lam} for a Fraction lam >= 0, by one min cut (the
    maximal maximiser of q|P(U)| - p|U|) -> bool (n,)."""
    lam = Fraction(lam)
    u = np.empty(G.n, np.uint8)
    if _load().orc_superlevel(G._h, mode, lam.numerator, lam.denominator, _p(u)) < 0:
        raise RuntimeError("oracle superlevel failed")
    return u.astype(bool)


def induced(G, keep):
    """Induced subgraph G[keep] -> (Graph on 0..k-1, ids (k,) of its vertices in G)."""
    keep = np.asarray(keep, bool)
    ids = np.flatnonzero(keep).astype(np.int64)
    new = np.full(G.n, -1, np.int64)
    new[ids] = np.arange(len(ids))
    u, v = G.edges()
    sel = keep[u] & keep[v]
    return Graph(len(ids), new[u[sel]].astype(np.int32), new[v[sel]].astype(np.int32)), ids


def top_levels(G, mode, lam):
    """Every LDS (mode 2) / LTDS (mode 3) of G with density >= lam > 0, by
    (density desc, min vertex asc), without the decomposition of all of G.

    U = {u : phi(u) >= lam} lies in the ceil(lam)-core K (phi <= core), and
    it is the maximal maximiser of q|P(U)| - p|U| over subsets of K as well
    as over all of V, so one min cut on G[K] finds it.  The nested maximal
    maximisers that define phi (Thm. 1 / Thm. cp) down to density lam lie in
    U, so the decomposition of G[U] gives phi_G on U.  An LDS of density
    rho >= lam is a component of {phi = rho} inside U with no neighbour of
    larger phi, and a neighbour outside U has phi < lam <= rho; so the rule
    of lds_from_phi applied to G[U] finds exactly the LDSs of G with density
    >= lam.  Returns (sets, |K|, |U|)."""
    lam = Fraction(lam)
    if lam <= 0:
        raise ValueError("lam must be > 0")
    k = -((-lam.numerator) // lam.denominator)  # ceil
    K = kcore(G, mode, k)
    GK, idK = induced(G, K)
    UK = superlevel(GK, mode, lam)
    GU, idU = induced(GK, UK)
    pn, pd = decompose(GU, mode)
    sets = []
    for vs, rho in lds_from_phi(GU, pn, pd):
        sets.append((np.sort(idK[idU[vs]]).astype(np.int32), rho))
    sets.sort(key=lambda t: (-t[1], int(t[0][0])))
    return sets, int(K.sum()), int(UK.sum())


def prune(G, mode, lo, hi):
    """Pruning (Alg. 3, Section 5.2) with bounds lo[u] <= phi(u) <= hi[u]
    (sequences of Fractions, by vertex): rule 1 (Cor. uv-prune) removes every
    vertex with a neighbour whose lower bound exceeds its upper bound; then
    rule 2 (Lemma uu-prune) removes, until nothing changes, every vertex whose
    core (tr-core) number in the subgraph induced by the remaining vertices
    is below its lower bound.  -> int8 (n,): 1 / 2 = removed by that rule,
    0 = kept.  Plain loops: small graphs only."""
    n = G.n
    rule = np.zeros(n, np.int8)
    u, v = G.edges()
    for a, b in zip(u.tolist(), v.tolist()):
        if lo[b] > hi[a]:
            rule[a] = 1
        if lo[a] > hi[b]:
            rule[b] = 1
    while True:
        keep = rule == 0
        sub, ids = induced(G, keep)
        core = core_numbers(sub, mode)
        changed = False
        for i, x in enumerate(ids.tolist()):
            if Fraction(int(core[i])) < lo[x]:
                rule[x] = 2
                changed = True
        if not changed:
            return rule
