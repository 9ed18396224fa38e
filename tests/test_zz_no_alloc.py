"""lds_frank_wolfe_noalloc, the entry point for callers that cannot allocate
device memory, against lds_frank_wolfe through the C ABI: the loads bit for
bit (exact numerators and the FP32 view), the gap within FP64 rounding (it is
formed on the device from the same exact sums), on two calls in a row, the
second on a smaller graph; its refusals; and, when the library holds no
device memory at the start (a fresh process), that it makes no device
allocation at all."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_helpers import announce

pytestmark = pytest.mark.gpu
lds = pytest.importorskip("paper_2504_10937_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)


class CountingAllocator:
    """the library's device allocations through torch's caching allocator,
    counted; active only if the library holds no device memory now"""

    def __init__(self):
        self.calls = 0
        dev = torch.cuda.current_device()

        def _alloc(nbytes, stream, ctx):
            self.calls += 1
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
            except Exception:
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        self.refs = (lds._ALLOC_FN(_alloc), lds._FREE_FN(_free))
        L = lds.load()
        st = L.lds_set_allocator(ctypes.cast(self.refs[0], ctypes.c_void_p), ctypes.cast(self.refs[1], ctypes.c_void_p),
                                 None)
        self.active = st == 0

    def close(self):
        if self.active:
            lds.load().lds_set_allocator(None, None, None)
            self.active = False


def reference(g, n, mode, iters):
    r = torch.empty(n, dtype=torch.float32, device="cuda")
    out = lds.lds_frank_wolfe(g, mode, iters, r_out=r, want_num=True, want_gap=True)
    torch.cuda.synchronize()
    return r.cpu().numpy(), out["num"], out["gap"]


def check_against(g, n, mode, iters, ref):
    r_ref, num_ref, gap_ref = ref
    r = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    gap = lds.lds_frank_wolfe_noalloc(g, mode, iters, r_out=r, want_gap=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.cpu().numpy(), r_ref)
    st = lds.lds_loads(g, mode, want_num=True)
    assert st["iters"] == iters
    np.testing.assert_array_equal(st["num"], num_ref)
    np.testing.assert_allclose(gap, gap_ref, rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("mode", [2, 3])
def test_noalloc_matches_frank_wolfe_two_calls(mode):
    announce("noalloc two calls", mode)
    counter = CountingAllocator()
    try:
        big = synth.powerlaw_planted(30000, 2.1, 10.0, 8, 20, 120, 0.3, seed=61)
        small = synth.powerlaw_planted(3000, 2.3, 8.0, 3, 10, 40, 0.5, seed=62)
        graphs = []
        for (n, s, d), iters in ((big, 120), (small, 45)):
            g = lds.lds_create_graph(n, s, d)
            graphs.append((g, n, iters, reference(g, n, mode, iters)))
        # two calls in a row, the second on the smaller graph with fewer iterations
        outs = []
        before = counter.calls
        for g, n, iters, _ in graphs:
            r = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
            outs.append((r, lds.lds_frank_wolfe_noalloc(g, mode, iters, r_out=r, want_gap=True)))
        if counter.active:
            assert counter.calls == before, "the no-allocation entry point allocated device memory"
        else:
            print("[note] device memory was live before the test: allocation count not checked", flush=True)
        torch.cuda.synchronize()
        for (g, n, iters, (r_ref, num_ref, gap_ref)), (r, gap) in zip(graphs, outs):
            np.testing.assert_array_equal(r.cpu().numpy(), r_ref)
            np.testing.assert_allclose(gap, gap_ref, rtol=1e-12, atol=0.0)
            st = lds.lds_loads(g, mode, want_num=True)
            assert st["iters"] == iters
            np.testing.assert_array_equal(st["num"], num_ref)
        # fewer iterations than the state holds, without the gap
        g, n, iters, _ = graphs[0]
        r = torch.empty(n, dtype=torch.float32, device="cuda")
        assert lds.lds_frank_wolfe_noalloc(g, mode, iters - 7, r_out=r) is None
        torch.cuda.synchronize()
        r_ref, _, _ = reference(g, n, mode, iters - 7)
        np.testing.assert_array_equal(r.cpu().numpy(), r_ref)
        for g, *_ in graphs:
            g.destroy()
    finally:
        counter.close()


def test_noalloc_refusals():
    announce("noalloc refusals")
    n, s, d = synth.powerlaw_planted(2000, 2.3, 8.0, 2, 10, 30, 0.5, seed=63)
    g = lds.lds_create_graph(n, s, d)
    # no FW state yet for either mode (and no triangles listed)
    for mode in (2, 3):
        with pytest.raises(lds.LdsError) as e:
            lds.lds_frank_wolfe_noalloc(g, mode, 10)
        assert e.value.status == 1
    lds.lds_frank_wolfe(g, 2, 10)
    lds.lds_frank_wolfe_noalloc(g, 2, 10)
    # more iterations than the state is sized for
    with pytest.raises(lds.LdsError) as e:
        lds.lds_frank_wolfe_noalloc(g, 2, 11)
    assert e.value.status == 1
    # beyond the fixed scratch with the gap: refused; without the gap: runs
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    limit = (1 << 19) // (4 * cus + 5)
    lds.lds_frank_wolfe(g, 2, limit + 1)
    with pytest.raises(lds.LdsError) as e:
        lds.lds_frank_wolfe_noalloc(g, 2, limit + 1, want_gap=True)
    assert e.value.status == 1
    gap = lds.lds_frank_wolfe_noalloc(g, 2, limit, want_gap=True)
    assert gap.shape == (limit,) and (gap >= 0).all()
    lds.lds_frank_wolfe_noalloc(g, 2, limit + 1)
    g.destroy()
