"""Python binding of liblds (include/lds.h): argument marshalling only.

Every computation runs in the gfx950 library; this module only converts
numpy arrays / torch tensors to pointers and statuses to exceptions.  The
library must be built (``python -m paper_2504_10937_amd.build`` or
``__graft_entry__.build()``); importing a function that needs it raises if it
is missing — there is no fallback path.

Names follow the C ABI: lds_create_graph, lds_frank_wolfe, ...
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblds.so")

LDS_EDGE = 2
LDS_TRIANGLE = 3
LDS_CLIQUE4 = 4
LDS_INPUT_DEVICE = 1
LDS_STRICT = 2
STATUS = {0: "LDS_OK", 1: "LDS_E_INVALID", 2: "LDS_E_NOMEM", 3: "LDS_E_DEVICE", 4: "LDS_E_OVERFLOW",
          5: "LDS_E_BUSY"}

_lib = None
# live native handles, released at interpreter exit while torch (whose
# allocator may own their memory) is still usable: servers, then batches,
# then graphs
_live = weakref.WeakSet()


@atexit.register
def _release_all():
    global _lib
    objs = list(_live)
    for cls in (Server, Batch, Graph):
        for o in objs:
            if isinstance(o, cls):
                o.destroy()
    _lib = None


class LdsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def load():
    """Load liblds.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblds.so is not built (run `python -m paper_2504_10937_amd.build`)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    st = ctypes.c_int
    sig = {
        "lds_last_error": (ctypes.c_char_p, []),
        "lds_set_allocator": (st, [vp, vp, vp]),
        "lds_create_graph": (st, [i64, i64, vp, vp, u32, vp, vp]),
        "lds_destroy_graph": (st, [vp]),
        "lds_graph_info": (st, [vp, vp, vp, vp, vp]),
        "lds_triangles": (st, [vp, vp, vp, i64, vp, vp]),
        "lds_cliques4": (st, [vp, vp, vp, i64, vp, vp]),
        "lds_frank_wolfe": (st, [vp, st, i32, vp, vp, vp, vp, vp]),
        "lds_frank_wolfe_noalloc": (st, [vp, st, i32, vp, vp, vp]),
        "lds_splits": (st, [vp, st, vp, vp, i64, vp, vp]),
        "lds_denominator": (u64, [st, i32]),
        "lds_fw_elapsed": (st, [vp, st, vp, vp]),
        "lds_sort_prefix": (st, [vp, st, vp, vp, vp, vp]),
        "lds_stable_groups": (st, [vp, st, vp, vp, vp, i64, vp, vp, vp]),
        "lds_sweep_info": (st, [vp, st, vp, vp, vp, vp, vp, vp]),
        "lds_sg_scan_info": (st, [vp, st, vp]),
        "lds_topk": (st, [vp, st, i32, i32, vp, vp]),
        "lds_result_free": (None, [vp]),
        "lds_prune": (st, [vp, st, i32, vp, vp, vp, vp]),
        "lds_loads": (st, [vp, st, vp, vp, vp, vp, vp, vp]),
        "lds_core_numbers": (st, [vp, st, vp, vp, vp]),
        "lds_fw_bounds": (st, [vp, st, vp, vp]),
        "lds_copy_bandwidth": (st, [vp, vp, ctypes.c_size_t, i32, vp, vp]),
        "lds_gather_rate": (st, [vp, i64, vp, i64, vp, i32, vp, vp]),
        "lds_tune_default": (None, [vp]),
        "lds_batch_create": (st, [vp, vp, vp, vp, i32, u32, vp, vp, vp]),
        "lds_batch_run": (st, [vp, vp]),
        "lds_batch_info": (st, [vp, vp, vp, vp, vp]),
        "lds_batch_destroy": (st, [vp]),
        "lds_batch_autotune": (st, [vp, vp, vp, i32, ctypes.c_char_p, i32, vp, vp, vp]),
        "lds_footprint": (st, [vp, st, i32, vp]),
        "lds_server_create": (st, [ctypes.c_size_t, i32, i32, vp]),
        "lds_server_submit": (st, [vp, vp, st, i32, i32, u64, ctypes.c_double]),
        "lds_server_poll": (st, [vp, vp, i32, ctypes.c_double, vp]),
        "lds_server_clock": (st, [vp, vp]),
        "lds_server_stats": (st, [vp, vp]),
        "lds_server_destroy": (st, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise LdsError(status, load().lds_last_error().decode(errors="replace"))


def _stream(stream):
    """hipStream_t of a torch stream (or the current torch stream)."""
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


class Graph:
    """Owning handle of an lds_graph."""

    def __init__(self, handle):
        self._h = handle
        _live.add(self)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lds_destroy_graph(self._h)
        self._h = None

    def __del__(self):
        self.destroy()

    def info(self):
        return lds_graph_info(self)


def lds_create_graph(n, src, dst, flags=0, stream=None):
    """Ingest an undirected graph from int32 endpoint arrays (numpy on the
    host, or torch tensors on the device)."""
    L = load()
    on_dev = hasattr(src, "is_cuda") and src.is_cuda
    if on_dev:
        import torch
        src = src.to(torch.int32).contiguous()
        dst = dst.to(torch.int32).contiguous()
        flags |= LDS_INPUT_DEVICE
        npairs = src.numel()
    else:
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        npairs = len(src)
    if npairs != (dst.numel() if on_dev else len(dst)):
        raise ValueError("src and dst differ in length")
    h = ctypes.c_void_p()
    _check(L.lds_create_graph(int(n), int(npairs), _ptr(src), _ptr(dst), flags, _stream(stream), ctypes.byref(h)))
    return Graph(h)


def lds_destroy_graph(g):
    g.destroy()


def lds_graph_info(g):
    n, m, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    b = ctypes.c_size_t()
    _check(load().lds_graph_info(g.handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(t), ctypes.byref(b)))
    return {"n": n.value, "m": m.value, "triangles": t.value, "device_bytes": b.value}


def lds_triangles(g, want_list=False, want_counts=False, stream=None):
    """List triangles on the device -> (|T|, (|T|,3) int32 or None, (n,) int64 or None)."""
    L = load()
    T = ctypes.c_int64()
    _check(L.lds_triangles(g.handle, ctypes.byref(T), None, 0, None, _stream(stream)))
    tri = cnt = None
    if want_list or want_counts:
        n = lds_graph_info(g)["n"]
        tri = np.empty((T.value, 3), np.int32) if want_list else None
        cnt = np.empty(n, np.int64) if want_counts else None
        _check(L.lds_triangles(g.handle, ctypes.byref(T), _ptr(tri), T.value, _ptr(cnt), _stream(stream)))
    return T.value, tri, cnt


def lds_cliques4(g, want_list=False, want_counts=False, stream=None):
    """List 4-cliques on the device -> (Q, (Q,4) int32 or None, (n,) int64 or None)."""
    L = load()
    Q = ctypes.c_int64()
    _check(L.lds_cliques4(g.handle, ctypes.byref(Q), None, 0, None, _stream(stream)))
    q = cnt = None
    if want_list or want_counts:
        n = lds_graph_info(g)["n"]
        q = np.empty((Q.value, 4), np.int32) if want_list else None
        cnt = np.empty(n, np.int64) if want_counts else None
        _check(L.lds_cliques4(g.handle, ctypes.byref(Q), _ptr(q), Q.value, _ptr(cnt), _stream(stream)))
    return Q.value, q, cnt


def lds_frank_wolfe(g, mode, iters, r_out=None, want_r64=False, want_num=False, want_gap=False, stream=None):
    """Run `iters` Frank-Wolfe iterations.  r_out: optional device float32
    tensor (n,).  Returns dict with 'r64', 'num', 'gap' as requested."""
    L = load()
    n = lds_graph_info(g)["n"]
    r64 = np.empty(n, np.float64) if want_r64 else None
    num = np.empty(n, np.uint64) if want_num else None
    gap = np.empty(iters, np.float64) if want_gap else None
    if r_out is not None and (r_out.numel() < n or not r_out.is_cuda):
        raise ValueError("r_out must be a device tensor with n elements")
    _check(L.lds_frank_wolfe(g.handle, mode, int(iters), _ptr(r_out), _ptr(r64), _ptr(num), _ptr(gap),
                             _stream(stream)))
    return {"r64": r64, "num": num, "gap": gap, "D": lds_denominator(mode, iters)}


def lds_frank_wolfe_noalloc(g, mode, iters, r_out=None, want_gap=False, stream=None):
    """lds_frank_wolfe without device allocation (the graph's FW state must
    already be sized for `iters`).  r_out: optional device float32 tensor
    (n,).  Returns the gap (iters,) or None."""
    L = load()
    n = lds_graph_info(g)["n"]
    if r_out is not None and (r_out.numel() < n or not r_out.is_cuda):
        raise ValueError("r_out must be a device tensor with n elements")
    gap = np.empty(iters, np.float64) if want_gap else None
    _check(L.lds_frank_wolfe_noalloc(g.handle, mode, int(iters), _ptr(r_out), _ptr(gap), _stream(stream)))
    return gap


def lds_splits(g, mode, stream=None):
    """Exact split numerators per incidence -> (verts (k,h) caller ids, num (k,))."""
    L = load()
    cnt = ctypes.c_int64()
    _check(L.lds_splits(g.handle, mode, None, None, 0, ctypes.byref(cnt), _stream(stream)))
    k = cnt.value
    verts = np.empty((k, mode), np.int32)
    num = np.empty(k, np.uint64)
    if k:
        _check(L.lds_splits(g.handle, mode, _ptr(verts), _ptr(num), k, ctypes.byref(cnt), _stream(stream)))
    return verts, num


def lds_denominator(mode, iters):
    return int(load().lds_denominator(mode, int(iters)))


def lds_sort_prefix(g, mode, stream=None):
    """The sort and prefix step of Alg. 2 on the last FW state -> (order (caller ids by position), E, inI)."""
    n = lds_graph_info(g)["n"]
    order = np.empty(n, np.int32)
    E = np.empty(n, np.int64)
    inI = np.empty(n, np.uint8)
    _check(load().lds_sort_prefix(g.handle, mode, _ptr(order), _ptr(E), _ptr(inI), _stream(stream)))
    return order, E, inI.astype(bool)


def _host_i64(n):
    """int64 output array of a device-to-host copy: page-locked (torch's
    caching host allocator) when a HIP device is present, so that the copy
    runs at link speed into pages that are reused, not faulted in anew."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.empty(n, dtype=torch.int64, pin_memory=True).numpy()
    except ImportError:
        pass
    return np.empty(n, np.int64)


def lds_stable_groups(g, mode, stream=None):
    """Alg. 2 stable groups -> (groups [(start, end)], lo (n,), hi (n,)) with
    lo/hi numerators over D (-1: no bounds), indexed by caller id."""
    n = lds_graph_info(g)["n"]
    ng = ctypes.c_int64()
    gs = np.empty(max(n, 1), np.int64)
    ge = np.empty(max(n, 1), np.int64)
    lo = _host_i64(n)
    hi = _host_i64(n)
    _check(load().lds_stable_groups(g.handle, mode, ctypes.byref(ng), _ptr(gs), _ptr(ge), len(gs), _ptr(lo), _ptr(hi),
                                    _stream(stream)))
    return [(int(gs[i]), int(ge[i])) for i in range(ng.value)], lo, hi


def lds_sg_scan_info(g, mode):
    """Profile of the last stable-group scan -> dict (groups, rounds,
    verifications, grid phases and microseconds per phase kind, positions
    searched, records walked, workgroups)."""
    out = np.zeros(14, np.int64)
    _check(load().lds_sg_scan_info(g.handle, mode, _ptr(out)))
    kinds = ("search", "update", "minmax", "accept")
    d = {"groups": int(out[0]), "rounds": int(out[1]), "verifications": int(out[2])}
    d.update({"grid_" + k: int(out[3 + i]) for i, k in enumerate(kinds)})
    d.update({"us_" + k: int(out[7 + i]) for i, k in enumerate(kinds)})
    d.update({"searched": int(out[11]), "walked": int(out[12]), "workgroups": int(out[13])})
    return d


def lds_fw_elapsed(g, mode):
    """(GPU ms of the sweep launches of the last FW run, number of launches)."""
    ms = ctypes.c_float()
    k = ctypes.c_int32()
    _check(load().lds_fw_elapsed(g.handle, mode, ctypes.byref(ms), ctypes.byref(k)))
    return ms.value, k.value


def lds_sweep_info(g, mode, stream=None):
    """Sweep shape -> dict(rows, slots, hub_rows, chunks, words)."""
    v = [ctypes.c_int64() for _ in range(5)]
    _check(load().lds_sweep_info(g.handle, mode, *[ctypes.byref(x) for x in v], _stream(stream)))
    return dict(zip(("rows", "slots", "hub_rows", "chunks", "words"), (x.value for x in v)))


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("vertices", ctypes.POINTER(ctypes.c_int32)), ("dens_num", ctypes.POINTER(ctypes.c_int64)),
                ("dens_den", ctypes.POINTER(ctypes.c_int64)), ("popped", ctypes.c_int64),
                ("refinements", ctypes.c_int64), ("flow_splits", ctypes.c_int64), ("maxflows", ctypes.c_int64),
                ("pruned", ctypes.c_int64), ("ms_copy", ctypes.c_double), ("ms_core", ctypes.c_double),
                ("ms_fw", ctypes.c_double), ("ms_prune", ctypes.c_double), ("ms_search", ctypes.c_double),
                ("refine_rounds", ctypes.c_int64)]


def _sets_of(r):
    from fractions import Fraction
    out = []
    if r.count > 0:
        off = np.ctypeslib.as_array(r.offsets, shape=(r.count + 1,)).copy()
        allv = np.ctypeslib.as_array(r.vertices, shape=(max(int(off[-1]), 1),))[:int(off[-1])].copy()
        for i in range(r.count):
            out.append((allv[off[i]:off[i + 1]].copy(), Fraction(int(r.dens_num[i]), int(r.dens_den[i]))))
    return out


def lds_topk(g, mode, k, iters, stream=None, with_stats=False):
    """Top-k LDS (mode 2) / LTDS (mode 3) -> list of (caller ids ascending,
    Fraction density), densest first; with_stats adds the search counters."""
    L = load()
    r = _Result()
    _check(L.lds_topk(g.handle, mode, int(k), int(iters), ctypes.byref(r), _stream(stream)))
    try:
        out = _sets_of(r)
        stats = {f: getattr(r, f) for f in ("popped", "refinements", "refine_rounds", "flow_splits", "maxflows",
                                              "pruned", "ms_copy", "ms_core", "ms_fw", "ms_prune", "ms_search")}
    finally:
        L.lds_result_free(ctypes.byref(r))
    return (out, stats) if with_stats else out


def lds_prune(g, mode, iters, stream=None):
    """Pruning (Alg. 3) as lds_topk runs it -> (rule (n,) int8 by caller id:
    1 / 2 = removed by rule 1 / 2, 0 = kept; pruned count; ms)."""
    n = lds_graph_info(g)["n"]
    rule = np.empty(max(n, 1), np.int8)
    cnt = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().lds_prune(g.handle, mode, int(iters), _ptr(rule), ctypes.byref(cnt), ctypes.byref(ms),
                            _stream(stream)))
    return rule[:n], cnt.value, ms.value


def lds_loads(g, mode, r_out=None, want_r64=False, want_num=False, want_gap=False, stream=None):
    """Current FW state of a mode (no run) -> dict(iters, r64?, num?, gap?)."""
    n = lds_graph_info(g)["n"]
    it = ctypes.c_int32()
    r64 = np.empty(n, np.float64) if want_r64 else None
    num = np.empty(n, np.uint64) if want_num else None
    _check(load().lds_loads(g.handle, mode, _ptr(r_out), _ptr(r64), _ptr(num), None, ctypes.byref(it),
                            _stream(stream)))
    out = {"iters": it.value}
    gap = np.empty(it.value, np.float64) if want_gap else None
    if want_gap:
        _check(load().lds_loads(g.handle, mode, None, None, None, _ptr(gap), None, _stream(stream)))
    out.update({k: v for k, v in (("r64", r64), ("num", num), ("gap", gap)) if v is not None})
    return out


def lds_fw_bounds(g, mode):
    """Lower bounds LB_i and certified gaps Gamma_i of the last FW run with
    the gap -> (lb (iters,), cert_gap (iters,))."""
    it = lds_loads(g, mode)["iters"]
    lb = np.empty(it, np.float64)
    cg = np.empty(it, np.float64)
    _check(load().lds_fw_bounds(g.handle, mode, _ptr(lb), _ptr(cg)))
    return lb, cg


def lds_gather_rate(idx, table, reps=5, stream=None):
    """Mean GPU ms of one pass of random 2-byte gathers table[idx[i]] by the
    library's gather kernel (idx: device int32 tensor of indices into table,
    a device uint16/int16 tensor)."""
    import torch
    if not (idx.is_cuda and table.is_cuda) or idx.dtype != torch.int32 or table.element_size() != 2:
        raise ValueError("idx must be a device int32 tensor and table a device 16-bit tensor")
    cus = torch.cuda.get_device_properties(idx.device).multi_processor_count
    sink = torch.empty(8 * 256 * cus, dtype=torch.int32, device=idx.device)
    ms = ctypes.c_float()
    _check(load().lds_gather_rate(_ptr(idx), idx.numel(), _ptr(table), table.numel(), _ptr(sink), int(reps),
                                  _stream(stream), ctypes.byref(ms)))
    return ms.value


def lds_copy_bandwidth(dst, src, reps=10, stream=None):
    """Mean GPU ms of one streaming copy src -> dst (device tensors of the
    same byte size, a multiple of 16) by the library's copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (dst.is_cuda and src.is_cuda):
        raise ValueError("dst and src must be device tensors of the same byte size")
    ms = ctypes.c_float()
    _check(load().lds_copy_bandwidth(_ptr(dst), _ptr(src), nbytes, int(reps), _stream(stream), ctypes.byref(ms)))
    return ms.value


def lds_core_numbers(g, mode, alive=None, stream=None):
    """Core (mode 2) / tr-core (mode 3) numbers by caller id -> int64 array;
    alive (n bools by caller id): those of the induced subgraph, -1 outside."""
    n = lds_graph_info(g)["n"]
    out = np.empty(n, np.int64)
    al = None if alive is None else np.ascontiguousarray(np.asarray(alive, dtype=bool).astype(np.uint8))
    if al is not None and al.shape != (n,):
        raise ValueError("alive must have n entries")
    _check(load().lds_core_numbers(g.handle, mode, _ptr(al), _ptr(out), _stream(stream)))
    return out


class LdsTune(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("lds_vertices", ctypes.c_int32),
                ("longest_first", ctypes.c_int32), ("max_kernel_cost", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


LDS_BATCH_GAP = 1


def lds_tune_default(**kw):
    t = LdsTune()
    load().lds_tune_default(ctypes.byref(t))
    for k, v in kw.items():
        setattr(t, k, v)
    return t


class Batch:
    """Owning handle of an lds_batch; keeps its graphs alive."""

    def __init__(self, handle, graphs, r_out):
        self._h = handle
        self._graphs = graphs
        self._r_out = r_out
        _live.add(self)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("batch destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lds_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        self.destroy()


def _batch_args(graphs, modes, iters):
    k = len(graphs)
    hs = (ctypes.c_void_p * max(k, 1))(*[g.handle for g in graphs])
    ms = (ctypes.c_int * max(k, 1))(*[int(m) for m in modes])
    its = (ctypes.c_int32 * max(k, 1))(*[int(i) for i in iters])
    return k, hs, ms, its


def lds_batch_create(graphs, modes, iters, r_out=None, gap=False, tune=None, stream=None):
    """Batch of FW runs (one per (graph, mode, iters)); r_out: optional list
    of device float tensors (or None entries) that receive the loads."""
    k, hs, ms, its = _batch_args(graphs, modes, iters)
    ro = None
    if r_out is not None:
        ro = (ctypes.c_void_p * max(k, 1))(*[(t.data_ptr() if t is not None else None) for t in r_out])
    out = ctypes.c_void_p()
    _check(load().lds_batch_create(hs, ms, its, ro, k, LDS_BATCH_GAP if gap else 0,
                                   ctypes.byref(tune) if tune is not None else None, _stream(stream),
                                   ctypes.byref(out)))
    return Batch(out.value, list(graphs), r_out)


def lds_batch_run(b, stream=None):
    _check(load().lds_batch_run(b.handle, _stream(stream)))


def lds_batch_info(b, want_ms=False):
    kg, pg = ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_float()
    t = LdsTune()
    _check(load().lds_batch_info(b.handle, ctypes.byref(kg), ctypes.byref(pg),
                                 ctypes.byref(ms) if want_ms else None, ctypes.byref(t)))
    out = {"kernel_graphs": kg.value, "plain_graphs": pg.value, "tune": t.as_dict()}
    if want_ms:
        out["kernel_ms"] = ms.value
    return out


def lds_batch_destroy(b):
    b.destroy()


def lds_batch_autotune(graphs, modes, iters, cache_path=None, reps=3, stream=None):
    """Fastest launch shape for this batch -> (LdsTune, best ms or -1 if cached)."""
    k, hs, ms, its = _batch_args(graphs, modes, iters)
    t = LdsTune()
    bm = ctypes.c_double()
    _check(load().lds_batch_autotune(hs, ms, its, k, cache_path.encode() if cache_path else None, int(reps),
                                     ctypes.byref(t), ctypes.byref(bm), _stream(stream)))
    return t, bm.value


class _Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("result", _Result),
                ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("error", ctypes.c_char * 160)]


class _ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_batch", ctypes.c_int64), ("pending", ctypes.c_int64), ("active", ctypes.c_int64),
                ("inflight_bytes", ctypes.c_size_t), ("peak_inflight_bytes", ctypes.c_size_t),
                ("batch_ms", ctypes.c_double)]


def lds_footprint(g, mode, iters):
    b = ctypes.c_size_t()
    _check(load().lds_footprint(g.handle, mode, int(iters), ctypes.byref(b)))
    return b.value


class Server:
    """Owning handle of an lds_server (continuous-batching query server)."""

    def __init__(self, handle):
        self._h = handle
        self._graphs = {}
        _live.add(self)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("server destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lds_server_destroy(self._h)
        self._h = None

    def __del__(self):
        self.destroy()


def lds_server_create(hbm_budget=0, max_slots=64, workers=8):
    out = ctypes.c_void_p()
    _check(load().lds_server_create(int(hbm_budget), int(max_slots), int(workers), ctypes.byref(out)))
    return Server(out.value)


def lds_server_submit(srv, g, mode, k, iters, tag, t_arrive=-1.0):
    srv._graphs[id(g)] = g  # keep the graph alive while the server may use it
    _check(load().lds_server_submit(srv.handle, g.handle, mode, int(k), int(iters), int(tag), float(t_arrive)))


def lds_server_poll(srv, max_n=256, wait_s=0.0):
    """-> list of dict(tag, status, sets, t_arrive, t_admit, t_done, error)."""
    L = load()
    arr = (_Completion * max(int(max_n), 1))()
    n = ctypes.c_int32()
    _check(L.lds_server_poll(srv.handle, arr, int(max_n), float(wait_s), ctypes.byref(n)))
    out = []
    for i in range(n.value):
        c = arr[i]
        d = {"tag": c.tag, "status": c.status, "t_arrive": c.t_arrive, "t_admit": c.t_admit, "t_done": c.t_done,
             "error": c.error.decode(errors="replace"), "sets": None}
        if c.status == 0:
            try:
                d["sets"] = _sets_of(c.result)
                d["stats"] = {f: getattr(c.result, f) for f in ("ms_copy", "ms_core", "ms_fw", "ms_prune",
                                                                "ms_search", "popped", "refinements")}
            finally:
                L.lds_result_free(ctypes.byref(c.result))
        out.append(d)
    return out


def lds_server_clock(srv):
    t = ctypes.c_double()
    _check(load().lds_server_clock(srv.handle, ctypes.byref(t)))
    return t.value


def lds_server_stats(srv):
    x = _ServerInfo()
    _check(load().lds_server_stats(srv.handle, ctypes.byref(x)))
    return {f: getattr(x, f) for f, _ in x._fields_}


def lds_server_destroy(srv):
    srv.destroy()


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None


def lds_set_allocator(use_torch=True):
    """Route the library's device allocations through PyTorch's caching
    allocator (use_torch=True) or back to hipMalloc/hipFree.  No graph may be
    alive when switching."""
    global _allocator_refs
    L = load()
    if not use_torch:
        _check(L.lds_set_allocator(None, None, None))
        _allocator_refs = None
        return
    import torch
    dev = torch.cuda.current_device()

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    refs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(L.lds_set_allocator(ctypes.cast(refs[0], ctypes.c_void_p), ctypes.cast(refs[1], ctypes.c_void_p), None))
    _allocator_refs = refs
