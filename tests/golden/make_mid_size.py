"""Write tests/golden/mid_size_<mode>.json: the oracle's Alg. 1 / Alg. 6 loads and
Alg. 2 (sort, prefix, index set I, stable groups and their bounds) on a
120,000-vertex power-law graph with planted blocks, both modes, at the
benchmark iteration counts (edges N = 100, triangles N = 200).

The graph is large enough that the library's sweep gathers the codes of
about a third of its vertices from memory (internal ids >= 77,824) and its
stable-group scan runs in its default
multi-workgroup shape (more than 16,384 vertices); the oracle's literal
ExtractSG is O(|I| (n + |P|)), minutes at this size, too slow for a test, so
its results are stored here as sha256 digests.

Calls only the oracle (oracle/) and the seeded generators (synth/).
Run: python tests/golden/make_mid_size.py [edge|triangle]  (~10 min per mode).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mid_size_%s.json")
GRAPH = dict(n=120000, beta=2.1, avg_deg=10.0, n_blocks=20, s_lo=30, s_hi=300, p_block=0.3, seed=31)
MODES = {"edge": (2, 100), "triangle": (3, 200)}


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def main():
    which = sys.argv[1:] or list(MODES)
    n, s, d = synth.powerlaw_planted(**GRAPH)
    G = oracle.Graph(n, s, d)
    for name in which:
        mode, iters = MODES[name]
        t0 = time.time()
        ref = oracle.fw_exact(G, mode, iters, with_gap=True)
        order, E, inI = oracle.sort_prefix(G, mode, ref["A"])
        print("[golden]", name, "fw + prefix", round(time.time() - t0, 1), "s; |I| =", int(inI.sum()), flush=True)
        groups, lo, hi = oracle.extract_sg(G, mode, ref["A"], ref["split"], ref["D"])
        print("[golden]", name, "stable groups", len(groups), round(time.time() - t0, 1), "s", flush=True)
        gs = np.array([a for a, _ in groups], np.int64)
        ge = np.array([b for _, b in groups], np.int64)
        out = {
            "source": "oracle/ only (tests/golden/make_mid_size.py); graph synth.powerlaw_planted(**graph)",
            "cite": "Alg. 1 / Alg. 6 (exact loads, gap); Alg. 2 with Def. 5 / Def. trsg (sort, prefix, I, stable "
                    "groups, bounds of Lemma phi-bounds)",
            "graph": GRAPH, "mode": mode, "iters": iters, "n": n, "m": G.m,
            "patterns": oracle.num_patterns(G, mode), "D": int(ref["D"]),
            "A_sha256": sha(ref["A"], "<u8"),
            "gap": [float(x) for x in ref["gap"]],
            "order_sha256": sha(order, "<i4"), "E_sha256": sha(E, "<i8"),
            "inI_sha256": sha(inI.astype(np.uint8), "u1"), "n_I": int(inI.sum()),
            "n_groups": len(groups), "gstart_sha256": sha(gs, "<i8"), "gend_sha256": sha(ge, "<i8"),
            "lo_sha256": sha(lo, "<i8"), "hi_sha256": sha(hi, "<i8"),
            "first_groups": [[int(a), int(b)] for a, b in groups[:20]],
        }
        with open(OUT % name, "w") as f:
            json.dump(out, f, indent=1)
        print("[golden] wrote", OUT % name, flush=True)


if __name__ == "__main__":
    main()
