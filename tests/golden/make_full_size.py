"""Write tests/golden/full_size.json: what the oracle alone computes for the
two full-size workloads that the benchmark reports (lds_large: edges,
N = 100; ltds_hk: triangles, N = 200).

Calls only the oracle (oracle/) and the seeded generators (synth/).  Stored
per workload:
  * sha256 of the exact load numerators A_u after N iterations of Alg. 1 /
    Alg. 6 (uint64 little-endian, by vertex id), and the duality gap of every
    iteration;
  * sha256 of Alg. 2's sort and prefix step on those loads: the order
    (int32), the prefix pattern counts E (int64) and the index set I (uint8);
  * the LDS (LTDS) sets of density >= lam, certified by the large-graph path
    (oracle.top_levels: k-core, one superlevel min cut, decomposition of the
    superlevel set).  lam is the largest prefix density of the oracle's own
    Alg. 2 order at N iterations (max_j E_j / j), a density some vertex set
    has, so the densest LDS is always among the sets.  The full decomposition
    of these graphs is out of the oracle's reach, so lower-density sets are
    not certified here.

Run: python tests/golden/make_full_size.py  (about 10 minutes, ~20 GB).
"""
import hashlib
import json
import os
import sys
import time
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def say(*a):
    print("[golden]", *a, flush=True)


def pick_lambda(E):
    """lam = the largest prefix density max_j E_j / j of Alg. 2's order: the
    density of an actual vertex set, so at most the largest density, and
    {phi >= lam} holds the densest subgraph; with converged loads it is close
    to that density, so the ceil(lam)-core is small"""
    j = np.arange(1, len(E) + 1, dtype=np.float64)
    d = E / j
    best = Fraction(0)
    for i in np.flatnonzero(d >= d.max() * (1 - 1e-9)):
        best = max(best, Fraction(int(E[i]), int(i) + 1))
    if best <= 0:
        raise RuntimeError("graph has no patterns")
    return best


def one(name):
    n, s, d, mode, iters, k = synth.workload(name)
    t0 = time.time()
    G = oracle.Graph(n, s, d)
    del s, d
    P = oracle.num_patterns(G, mode)
    say(name, "n", n, "m", G.m, "patterns", P)
    ref = oracle.fw_exact(G, mode, iters, with_gap=True, with_split=False)
    say(name, "fw done", round(time.time() - t0, 1), "s")
    order, E, inI = oracle.sort_prefix(G, mode, ref["A"])
    say(name, "sort/prefix done", round(time.time() - t0, 1), "s")
    lam = pick_lambda(E)
    sets, K, U = oracle.top_levels(G, mode, lam)
    say(name, "top levels at", lam, ":", len(sets), "sets, core", K, "superlevel", U, round(time.time() - t0, 1), "s")
    return {
        "workload": name, "mode": mode, "iters": iters, "n": n, "m": G.m, "patterns": P,
        "D": int(ref["D"]),
        "A_sha256": sha(ref["A"], "<u8"),
        "A_sum": int(ref["A"].sum(dtype=np.uint64)),
        "gap": [float(x) for x in ref["gap"]],
        "order_sha256": sha(order, "<i4"),
        "E_sha256": sha(E, "<i8"),
        "inI_sha256": sha(inI.astype(np.uint8), "u1"),
        "n_I": int(inI.sum()),
        "lambda": [lam.numerator, lam.denominator],
        "kcore_size": K, "superlevel_size": U,
        "sets": [{"size": len(v), "rho": [r.numerator, r.denominator], "vertices": [int(x) for x in v]}
                 for v, r in sets],
    }


def main():
    out = {
        "source": "oracle/ only (tests/golden/make_full_size.py); inputs from synth.workload",
        "cite": {
            "A, gap": "Alg. 1 (edges, Eq. cp) and Alg. 6 (triangles, Eq. trcp) in exact rational form; gap = "
                      "2 (sum r^2 - sum_patterns min r) at r^(i-1)",
            "order, E, I": "Alg. 2 (ExtractSG), sort by r and prefix densities, ties to the larger index (Section 5.1)",
            "sets": "Problem LDS (Section 3) / Problem LTDS (Section 6.1): LDSs from compact numbers (Thm. 1, "
                    "Thm. cnltds) restricted to density >= lambda",
        },
    }
    names = sys.argv[1:] or ["lds_large", "ltds_hk"]
    if os.path.exists(OUT):
        with open(OUT) as f:
            out.update({k: v for k, v in json.load(f).items() if k in ("lds_large", "ltds_hk")})
    for name in names:
        out[name] = one(name)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1)
        say("wrote", OUT)


if __name__ == "__main__":
    main()
