"""Batched Frank-Wolfe (one persistent hipGraph-captured launch over many
graphs) against per-graph runs: the same exact loads, split numerators,
gap values and stable groups, for every launch shape the autotuner may pick,
and against the oracle on a few members."""
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


def members(count, start=0):
    out = []
    for i in range(start, start + count):
        n, s, d = synth.batch_member(i)
        mode = 2 if i % 2 == 0 else 3
        out.append((n, s, d, mode, 100 if mode == 2 else 200))
    return out


def per_graph(ms, gap=True):
    ref = []
    for n, s, d, mode, it in ms:
        g = lds.lds_create_graph(n, s, d)
        o = lds.lds_frank_wolfe(g, mode, it, want_num=True, want_gap=gap)
        ref.append((o["num"], o["gap"], lds.lds_splits(g, mode)))
    return ref


def check_same(gs, ms, ref, gap=True):
    for g, (n, s, d, mode, it), (num, gp, sp) in zip(gs, ms, ref):
        out = lds.lds_loads(g, mode, want_num=True, want_gap=gap)
        assert out["iters"] == it
        np.testing.assert_array_equal(out["num"], num)
        if gap:
            np.testing.assert_array_equal(out["gap"], gp)
        v, a = lds.lds_splits(g, mode)
        np.testing.assert_array_equal(v, sp[0])
        np.testing.assert_array_equal(a, sp[1])


TUNES = [
    dict(),
    dict(threads=256, wg_per_cu=2),
    dict(threads=512, wg_per_cu=1, longest_first=0),
    dict(lds_vertices=0),                 # keys in device memory
    dict(lds_vertices=600),               # mixed: small graphs in LDS, larger in memory
    dict(max_kernel_cost=200000),         # larger graphs run one by one
]


@pytest.mark.parametrize("tune", range(len(TUNES)))
def test_batch_matches_per_graph(tune):
    announce("batch vs per-graph", TUNES[tune])
    ms = members(24)
    ref = per_graph(ms)
    gs = [lds.lds_create_graph(n, s, d) for n, s, d, _, _ in ms]
    t = lds.lds_tune_default(**TUNES[tune])
    b = lds.lds_batch_create(gs, [m[3] for m in ms], [m[4] for m in ms], gap=True, tune=t)
    lds.lds_batch_run(b)
    info = lds.lds_batch_info(b, want_ms=True)
    assert info["kernel_graphs"] + info["plain_graphs"] == len(ms)
    check_same(gs, ms, ref)


def test_batch_replays_and_r_out():
    """Replays of the captured graph, with eager work between them, all give
    the per-graph result; r_out receives the float loads."""
    announce("batch replays")
    ms = members(16, start=40)
    ref = per_graph(ms, gap=False)
    gs = [lds.lds_create_graph(n, s, d) for n, s, d, _, _ in ms]
    rs = [torch.full((n,), -1.0, device="cuda") for n, *_ in ms]
    b = lds.lds_batch_create(gs, [m[3] for m in ms], [m[4] for m in ms], r_out=rs)
    for rep in range(3):
        lds.lds_batch_run(b)
        torch.cuda.synchronize()
        check_same(gs, ms, ref, gap=False)
        for r, (num, _, _), (n, s, d, mode, it) in zip(rs, ref, ms):
            want = (num.astype(np.float64) / lds.lds_denominator(mode, it)).astype(np.float32)
            np.testing.assert_array_equal(r.cpu().numpy(), want)
            r.fill_(-1.0)
        # eager work on the same graphs between replays
        lds.lds_frank_wolfe(gs[0], ms[0][3], 3)
        torch.cuda.synchronize()


def test_batch_against_oracle():
    announce("batch vs oracle")
    ms = members(6, start=100)
    gs = [lds.lds_create_graph(n, s, d) for n, s, d, _, _ in ms]
    b = lds.lds_batch_create(gs, [m[3] for m in ms], [m[4] for m in ms], gap=True)
    lds.lds_batch_run(b)
    for g, (n, s, d, mode, it) in zip(gs, ms):
        G = oracle.Graph(n, s, d)
        ref = oracle.fw_exact(G, mode, it, with_split=False)
        out = lds.lds_loads(g, mode, want_num=True, want_gap=True)
        np.testing.assert_array_equal(out["num"], ref["A"])
        np.testing.assert_allclose(out["gap"], ref["gap"], rtol=1e-12, atol=0)


def test_batch_then_stable_groups_and_topk():
    """State left by the batch feeds the stable-group pass unchanged."""
    announce("batch then stable groups")
    ms = members(8, start=200)
    gs = [lds.lds_create_graph(n, s, d) for n, s, d, _, _ in ms]
    b = lds.lds_batch_create(gs, [m[3] for m in ms], [m[4] for m in ms])
    lds.lds_batch_run(b)
    for g, (n, s, d, mode, it) in zip(gs, ms):
        groups, lo, hi = lds.lds_stable_groups(g, mode)
        h = lds.lds_create_graph(n, s, d)
        lds.lds_frank_wolfe(h, mode, it)
        g2, lo2, hi2 = lds.lds_stable_groups(h, mode)
        assert groups == g2
        np.testing.assert_array_equal(lo, lo2)
        np.testing.assert_array_equal(hi, hi2)


def test_batch_degenerate_members():
    announce("batch degenerate")
    e = np.zeros(0, np.int32)
    inputs = [
        (7, e, e),                                                                  # no edges
        (4, np.array([0, 1, 2], np.int32), np.array([1, 2, 3], np.int32)),          # a path: no triangles
        (3, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32)),          # one triangle
        (0, e, e),                                                                  # no vertices
    ]
    cases = [(0, 2, 5), (1, 2, 7), (1, 3, 9), (2, 2, 0), (2, 3, 4), (3, 3, 3)]
    made = {}
    graphs = []
    for k, mode, it in cases:
        if k not in made:
            made[k] = lds.lds_create_graph(*inputs[k])
        graphs.append(made[k])
    b = lds.lds_batch_create(graphs, [c[1] for c in cases], [c[2] for c in cases], gap=True)
    lds.lds_batch_run(b)
    for g, (k, mode, it) in zip(graphs, cases):
        out = lds.lds_loads(g, mode, want_num=True, want_gap=True)
        ref = lds.lds_frank_wolfe(lds.lds_create_graph(*inputs[k]), mode, it, want_num=True, want_gap=True)
        np.testing.assert_array_equal(out["num"], ref["num"])
        np.testing.assert_array_equal(out["gap"], ref["gap"])
    # an empty batch runs; a (graph, mode) pair may not appear twice
    lds.lds_batch_run(lds.lds_batch_create([], [], []))
    with pytest.raises(lds.LdsError):
        lds.lds_batch_create([made[2], made[2]], [2, 2], [3, 3])


def test_autotune_cache(tmp_path):
    announce("autotune cache")
    ms = members(32, start=300)
    gs = [lds.lds_create_graph(n, s, d) for n, s, d, _, _ in ms]
    modes, iters = [m[3] for m in ms], [m[4] for m in ms]
    cache = str(tmp_path / "tune.json")
    t, best = lds.lds_batch_autotune(gs, modes, iters, cache_path=cache, reps=1)
    assert best > 0 and t.threads in (256, 512, 1024)
    t2, best2 = lds.lds_batch_autotune(gs, modes, iters, cache_path=cache, reps=1)
    assert best2 == -1 and t2.as_dict() == t.as_dict()
    ref = per_graph(ms, gap=False)
    b = lds.lds_batch_create(gs, modes, iters, tune=t2)
    lds.lds_batch_run(b)
    check_same(gs, ms, ref, gap=False)
