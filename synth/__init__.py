"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

Holds no arithmetic of the densest-subgraph method: it only builds edge lists
(COO pairs, possibly with duplicates and random orientation, never with
self-loops) and query streams, from the C generators in ``gen.c``.

Workload recipes (the paper's datasets are absent, so these synthetic graphs
stand in for them with power-law degrees and planted dense blocks):

* ``lds_small``  Chung-Lu beta=2.3, n=2000, mean degree 8, 10 planted
  G(s,0.5) blocks, s in [20,60]; LDS, N=200, k=5.
* ``lds_large``  Chung-Lu beta=2.1, n=4M, mean degree 30 (~60M edges),
  200 planted G(s,0.3) blocks, s in [50,2000]; LDS, N=100, k=10.
* ``ltds_hk``    Holme-Kim n=1M, 20 edges per vertex, triad formation 0.6;
  LTDS, N=200, k=10.
* ``batch``      4096 members, n log-uniform in [50,5000] (seed 1000+g).
* ``pool``       64 members, n lognormal(median 1e4, sigma 1.5) clipped to
  [50, 2M], member 0 pinned at 2M; Poisson query stream at 200 QPS.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build():
    """Compile the generator library in-tree (gcc, C11)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", src, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    vp, i64, i32, f64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64
    lib.synth_powerlaw_planted.restype = vp
    lib.synth_powerlaw_planted.argtypes = [i64, f64, f64, i32, i32, i32, f64, u64]
    lib.synth_holme_kim.restype = vp
    lib.synth_holme_kim.argtypes = [i64, i32, f64, u64]
    lib.synth_erdos_renyi.restype = vp
    lib.synth_erdos_renyi.argtypes = [i64, f64, u64]
    lib.synth_batch_member.restype = vp
    lib.synth_batch_member.argtypes = [i64, u64, f64, f64]
    lib.synth_pool_member.restype = vp
    lib.synth_pool_member.argtypes = [i64, u64, f64, f64, i64]
    lib.synth_num_vertices.restype = i64
    lib.synth_num_vertices.argtypes = [vp]
    lib.synth_num_pairs.restype = i64
    lib.synth_num_pairs.argtypes = [vp]
    lib.synth_copy.restype = None
    lib.synth_copy.argtypes = [vp, vp, vp]
    lib.synth_free.restype = None
    lib.synth_free.argtypes = [vp]
    lib.synth_queries.restype = None
    lib.synth_queries.argtypes = [i64, f64, i32, i32, u64, vp, vp, vp, vp]
    _lib = lib
    return lib


def _take(h):
    lib = _load()
    if not h:
        raise RuntimeError("synth: generator failed (bad arguments or out of memory)")
    try:
        n = lib.synth_num_vertices(h)
        m = lib.synth_num_pairs(h)
        src = np.empty(m, dtype=np.int32)
        dst = np.empty(m, dtype=np.int32)
        lib.synth_copy(h, src.ctypes.data, dst.ctypes.data)
    finally:
        lib.synth_free(h)
    return int(n), src, dst


def powerlaw_planted(n, beta, avg_deg, n_blocks=0, s_lo=2, s_hi=2, p_block=0.0, seed=0):
    """Chung-Lu power-law background plus planted G(s,p) blocks -> (n, src, dst)."""
    lib = _load()
    return _take(lib.synth_powerlaw_planted(n, beta, avg_deg, n_blocks, s_lo, s_hi, p_block, seed))


def holme_kim(n, mper, p_triad, seed=0):
    """Holme-Kim preferential attachment with triad formation -> (n, src, dst)."""
    return _take(_load().synth_holme_kim(n, mper, p_triad, seed))


def erdos_renyi(n, p, seed=0):
    """G(n,p) (n <= 1e5) -> (n, src, dst)."""
    return _take(_load().synth_erdos_renyi(n, p, seed))


def barabasi_albert(n, m, seed=0):
    """Barabasi-Albert preferential attachment with m edges per new vertex
    (Holme-Kim with triad-formation probability 0) -> (n, src, dst)."""
    return holme_kim(n, m, 0.0, seed=seed)


def batch_member(index, base_seed=1000, n_lo=50.0, n_hi=5000.0):
    """Member `index` of the uneven batch (seed base_seed+index) -> (n, src, dst)."""
    return _take(_load().synth_batch_member(index, base_seed, n_lo, n_hi))


def pool_member(index, base_seed=5, median=1.0e4, sigma=1.5, n_max=2_000_000):
    """Member `index` of the resident serving pool -> (n, src, dst)."""
    return _take(_load().synth_pool_member(index, base_seed, median, sigma, n_max))


def queries(count, qps=200.0, pool=64, kmax=10, seed=5):
    """Poisson query stream -> dict of arrays (t_arrive s, graph, mode 2|3, k)."""
    lib = _load()
    t = np.empty(count, dtype=np.float64)
    g = np.empty(count, dtype=np.int32)
    md = np.empty(count, dtype=np.int32)
    k = np.empty(count, dtype=np.int32)
    lib.synth_queries(count, qps, pool, kmax, seed, t.ctypes.data, g.ctypes.data, md.ctypes.data, k.ctypes.data)
    return {"t_arrive": t, "graph": g, "mode": md, "k": k}


# Named workloads: (generator, kwargs, mode, iterations, k)
WORKLOADS = {
    "lds_small": (powerlaw_planted, dict(n=2000, beta=2.3, avg_deg=8.0, n_blocks=10, s_lo=20, s_hi=60,
                                         p_block=0.5, seed=1), 2, 200, 5),
    "lds_large": (powerlaw_planted, dict(n=4_000_000, beta=2.1, avg_deg=30.0, n_blocks=200, s_lo=50,
                                         s_hi=2000, p_block=0.3, seed=2), 2, 100, 10),
    "ltds_hk": (holme_kim, dict(n=1_000_000, mper=20, p_triad=0.6, seed=3), 3, 200, 10),
}
# 4-clique program (h = 4): power-law background with 200 planted G(s, 0.5)
# blocks, s in [20, 120]; 1.66e8 4-cliques
WORKLOADS["clique4_pl"] = (powerlaw_planted, dict(n=1_000_000, beta=2.2, avg_deg=10.0, n_blocks=200, s_lo=20,
                                                  s_hi=120, p_block=0.5, seed=4), 4, 100, 0)
# the density sweep of the scalability experiment (Section 8): n = 1M, density
# |E|/|V| = 2, 4, ..., 12, LDScvx with the default N = 100 and k = 5
for _d in range(2, 13, 2):
    WORKLOADS["ba_d%d" % _d] = (barabasi_albert, dict(n=1_000_000, m=_d, seed=100 + _d), 2, 100, 5)


def workload(name):
    """Return (n, src, dst, mode, iterations, k) for a named workload."""
    fn, kw, mode, iters, k = WORKLOADS[name]
    n, s, d = fn(**kw)
    return n, s, d, mode, iters, k
