"""Serving loop: queries admitted by memory budget and slots, batched FW
launches, verification overlapped on worker threads.  Each result must be
the one lds_topk gives for the same (graph, mode, k, iters) alone, whatever
else is in flight; admission must respect the budget."""
import time

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


def pool(count, start=0):
    return [synth.batch_member(i, base_seed=5000) for i in range(start, start + count)]


def alone(inputs, queries):
    """lds_topk on fresh graphs, one query at a time"""
    out = {}
    for tag, (gi, mode, k, it) in queries.items():
        g = lds.lds_create_graph(*inputs[gi])
        out[tag] = lds.lds_topk(g, mode, k, it)
    return out


def same(got, ref):
    assert len(got) == len(ref)
    for (a, x), (b, y) in zip(got, ref):
        assert x == y
        np.testing.assert_array_equal(a, b)


def drain(srv, count, timeout=120.0):
    done = {}
    t0 = time.time()
    while len(done) < count:
        assert time.time() - t0 < timeout, "server did not finish"
        for c in lds.lds_server_poll(srv, 64, 0.5):
            done[c["tag"]] = c
    return done


def make_queries(n_graphs, count, seed):
    rng = np.random.default_rng(seed)
    q = {}
    for tag in range(count):
        mode = int(rng.choice([2, 3]))
        q[tag] = (int(rng.integers(n_graphs)), mode, int(rng.integers(1, 11)), 40 if mode == 2 else 60)
    return q


def test_results_same_alone_and_in_the_mix():
    announce("server mix")
    inputs = pool(10)
    queries = make_queries(len(inputs), 60, seed=1)
    ref = alone(inputs, queries)
    gs = [lds.lds_create_graph(*x) for x in inputs]
    srv = lds.lds_server_create(0, max_slots=16, workers=4)
    for tag, (gi, mode, k, it) in queries.items():
        lds.lds_server_submit(srv, gs[gi], mode, k, it, tag)
        if tag % 7 == 0:
            time.sleep(0.002)  # some arrive while others are on the GPU
    done = drain(srv, len(queries))
    st = lds.lds_server_stats(srv)
    lds.lds_server_destroy(srv)
    assert st["completed"] == len(queries) and st["batches"] >= 1
    for tag, c in done.items():
        assert c["status"] == 0, c["error"]
        assert c["t_arrive"] <= c["t_admit"] <= c["t_done"]
        same(c["sets"], ref[tag])


def test_against_oracle_in_the_mix():
    announce("server vs oracle")
    inputs = pool(4, start=20)
    queries = {t: (t % 4, 2 if t < 4 else 3, 5, 50) for t in range(8)}
    gs = [lds.lds_create_graph(*x) for x in inputs]
    srv = lds.lds_server_create(0, max_slots=8, workers=2)
    for tag, (gi, mode, k, it) in queries.items():
        lds.lds_server_submit(srv, gs[gi], mode, k, it, tag)
    done = drain(srv, len(queries))
    lds.lds_server_destroy(srv)
    for tag, (gi, mode, k, it) in queries.items():
        G = oracle.Graph(*inputs[gi])
        ref = oracle.top_k(G, mode, k)
        same(done[tag]["sets"], ref)


def test_admission_by_memory_budget():
    """A budget that holds one query at a time still gives every result; a
    query larger than the budget is refused with LDS_E_NOMEM."""
    announce("server admission")
    inputs = pool(6, start=40)
    queries = make_queries(len(inputs), 24, seed=2)
    ref = alone(inputs, queries)
    gs = [lds.lds_create_graph(*x) for x in inputs]
    for g in gs:
        lds.lds_triangles(g)
    fps = [lds.lds_footprint(gs[gi], mode, it) for gi, mode, k, it in queries.values()]
    budget = max(fps)
    srv = lds.lds_server_create(budget, max_slots=64, workers=4)
    for tag, (gi, mode, k, it) in queries.items():
        lds.lds_server_submit(srv, gs[gi], mode, k, it, tag)
    # one query that cannot fit
    big = synth.batch_member(0, base_seed=7000, n_lo=4000, n_hi=5000)
    gb = lds.lds_create_graph(*big)
    big_iters = 200
    while lds.lds_footprint(gb, 2, big_iters) <= budget:
        big_iters *= 2
    lds.lds_server_submit(srv, gb, 2, 3, big_iters, 999)
    done = drain(srv, len(queries) + 1)
    st = lds.lds_server_stats(srv)
    lds.lds_server_destroy(srv)
    assert st["peak_inflight_bytes"] <= budget
    for tag, c in done.items():
        if tag == 999:
            continue
        assert c["status"] == 0, c["error"]
        same(c["sets"], ref[tag])
    assert done[999]["status"] == 2


@pytest.mark.parametrize("big", [False, True])
def test_same_graph_queries_run_at_once(big):
    """Queries on one graph and mode run at once, each on its own view of the
    graph (its own FW and stable-group state): results equal lds_topk run
    alone, and queries on the same (graph, mode) overlap in time.  big: a
    graph whose FW runs on the worker's own launches instead of the batched
    kernel."""
    announce("server same graph", big)
    inputs = [synth.powerlaw_planted(20000, 2.2, 10.0, 6, 20, 80, 0.4, seed=63)] if big else pool(1, start=60)
    g = lds.lds_create_graph(*inputs[0])
    queries = {t: (0, 2 + t % 2, 1 + t % 10, 20 + 3 * t) for t in range(16)}
    ref = alone(inputs, queries)
    srv = lds.lds_server_create(0, max_slots=16, workers=6)
    for tag, (gi, mode, k, it) in queries.items():
        lds.lds_server_submit(srv, g, mode, k, it, tag)
    done = drain(srv, len(queries))
    lds.lds_server_destroy(srv)
    for tag, c in done.items():
        assert c["status"] == 0, c["error"]
        same(c["sets"], ref[tag])
    # some pair of queries on the same (graph, mode) was in flight together
    spans = [(c["t_admit"], c["t_done"], queries[t][1]) for t, c in done.items()]
    assert any(a0 < b1 and b0 < a1 and ma == mb
               for i, (a0, a1, ma) in enumerate(spans) for (b0, b1, mb) in spans[i + 1:])
    # the graph itself is untouched and usable
    same(lds.lds_topk(g, 2, 3, 30), alone(inputs, {0: (0, 2, 3, 30)})[0])


def test_destroy_with_queued_queries():
    announce("server destroy")
    inputs = pool(3, start=80)
    gs = [lds.lds_create_graph(*x) for x in inputs]
    srv = lds.lds_server_create(0, max_slots=1, workers=1)
    for tag in range(20):
        lds.lds_server_submit(srv, gs[tag % 3], 2, 3, 30, tag)
    lds.lds_server_destroy(srv)  # drops the queued ones, finishes the admitted one
    # the graphs are usable afterwards
    assert len(lds.lds_topk(gs[0], 2, 3, 30)) >= 1
