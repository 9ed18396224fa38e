"""A process that leaves graphs, a batch and a server alive when it exits,
with the library's memory coming from torch's caching allocator, exits
cleanly: the binding releases every native handle at interpreter exit,
servers first, while torch is still usable."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
import numpy as np, torch
import paper_2504_10937_amd as lds, synth
lds.lds_set_allocator(True)
gs = []
for i in range(6):
    n, s, d = synth.batch_member(i)
    gs.append(lds.lds_create_graph(n, s, d))
b = lds.lds_batch_create(gs[:3], [2, 3, 2], [20, 20, 20])
lds.lds_batch_run(b)
srv = lds.lds_server_create(0, max_slots=8, workers=4)
for i, g in enumerate(gs):
    lds.lds_server_submit(srv, g, 2, 2, 20, i)
got = 0
while got < 6:
    got += len(lds.lds_server_poll(srv, 16, 1.0))
print("child done", flush=True)
"""


def test_exit_with_live_handles():
    print("[case] exit with live handles", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD % ROOT], capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "child done" in r.stdout
