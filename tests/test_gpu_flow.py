"""The device push-relabel (the min cuts of IsDensest on large vertex
networks): forced onto every vertex network, on one workgroup and on grids
of several, the top-k answers stay exactly the oracle's (the min cut decides
every IsDensest / IsLDS step, so a wrong flow or cut changes the answer)."""
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

WIDTHS = ["1", "3", "16"]


def same(got, ref):
    assert len(got) == len(ref)
    for (a, x), (b, y) in zip(got, ref):
        assert x == y
        np.testing.assert_array_equal(a, b)


def on_device(monkeypatch, width):
    monkeypatch.setenv("LDS_FLOW_GPU_MIN", "0")
    monkeypatch.setenv("LDS_FLOW_GPU_WG", width)


@pytest.mark.parametrize("width", WIDTHS)
@pytest.mark.parametrize("d", [2, 6])
def test_barabasi_albert(d, width, monkeypatch):
    on_device(monkeypatch, width)
    n, s, t = synth.barabasi_albert(20000, d, seed=7 + d)
    announce("device flow ba", d, width)
    G = oracle.Graph(n, s, t)
    g = lds.lds_create_graph(n, s, t)
    same(lds.lds_topk(g, 2, 5, 100), oracle.top_k(G, 2, 5))


@pytest.mark.parametrize("width", WIDTHS)
def test_holme_kim_all_sets(width, monkeypatch):
    on_device(monkeypatch, width)
    n, s, d = synth.holme_kim(3000, 5, 0.6, seed=4)
    announce("device flow holme-kim", width)
    G = oracle.Graph(n, s, d)
    g = lds.lds_create_graph(n, s, d)
    same(lds.lds_topk(g, 2, 1000, 100), oracle.top_k(G, 2, 1000))


@pytest.mark.parametrize("width", WIDTHS)
def test_powerlaw_planted_all_sets(width, monkeypatch):
    on_device(monkeypatch, width)
    n, s, d = synth.powerlaw_planted(4000, 2.2, 10.0, n_blocks=12, s_lo=15, s_hi=80, p_block=0.4, seed=7)
    announce("device flow powerlaw", width)
    G = oracle.Graph(n, s, d)
    g = lds.lds_create_graph(n, s, d)
    same(lds.lds_topk(g, 2, 100000, 60), oracle.top_k(G, 2, 100000))


@pytest.mark.parametrize("seed", range(6))
def test_tiny_against_brute_force(seed, monkeypatch):
    on_device(monkeypatch, "2")
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(4, 13))
    n, s, d = synth.erdos_renyi(n, float(rng.uniform(0.25, 0.7)), seed=400 + seed)
    announce("device flow tiny", seed, n, len(s))
    G = oracle.Graph(n, s, d)
    _, sets = oracle.brute(G, 2)
    g = lds.lds_create_graph(n, s, d)
    same(lds.lds_topk(g, 2, 1000, 10), sets)
