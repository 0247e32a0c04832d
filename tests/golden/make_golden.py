"""Write oracle-computed expected counts for full-size workloads.

Calls only the oracle (and the seeded input generators).  Usage:
    python tests/golden/make_golden.py chung_lu_1m [threads]
writes tests/golden/chung_lu_1m_seed0.json with n, m, the oracle's 128-bit
sums, the 45 non-induced and the 45 induced counts (decimal strings).
The 1M-vertex graph takes about 50 minutes on 8 host cores.
    python tests/golden/make_golden.py batch_10k [threads]
writes tests/golden/batch_10k_seed0.txt: for each of the 10^4 graphs of the
batched workload (seed 0) one line "index n m digest", digest = the first 16
hex digits of the SHA-256 of the 45 induced counts written as decimal
numbers joined by commas (about 5 minutes on 8 host cores).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import patterns as pat  # noqa: E402

WORKLOADS = {
    "chung_lu_1m": (lambda: synth.chung_lu_1m(0), "chung_lu_1m_seed0.json",
                    "Chung-Lu n=1e6 gamma=2.1 mean degree 20 max expected degree 1e4, seed 0"),
}


def count_digest(counts):
    """First 16 hex digits of the SHA-256 of the counts as comma-joined decimals."""
    import hashlib
    return hashlib.sha256(",".join(str(int(x)) for x in counts).encode()).hexdigest()[:16]


def batch_10k(threads):
    specs = synth.batch_specs(10_000, 0)
    t0 = time.time()
    lines = ["# batched workload, 10^4 graphs (synth.batch_specs(10000, 0)): index n m digest of the 45 induced "
             "counts (oracle.count, k = 5; see make_golden.py)"]
    for i, sp in enumerate(specs):
        g = synth.from_spec(sp)
        lines.append("%d %d %d %s" % (i, g.n, g.m, count_digest(oracle.count(g, 5, threads=threads))))
    with open(os.path.join(HERE, "batch_10k_seed0.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote batch_10k_seed0.txt in %.0f s" % (time.time() - t0))


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "chung_lu_1m"
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    if name == "batch_10k":
        batch_10k(threads)
        return
    make, fname, desc = WORKLOADS[name]
    g = make()
    t0 = time.time()
    S = oracle.sums(g, 5, threads=threads)
    secs = time.time() - t0
    non = oracle.noninduced_from_sums(S, 4) + oracle.noninduced_from_sums(S, 5)
    ind = pat.induced_from_noninduced(4, non[:11]) + pat.induced_from_noninduced(5, non[11:])
    out = {
        "workload": desc, "n": g.n, "m": g.m,
        "oracle_seconds": secs, "oracle_threads": threads,
        "sums": {k: str(v) for k, v in S.items()},
        "noninduced": [str(x) for x in non],
        "counts": [str(x) for x in ind],
        "names": pat.ALL_NAMES,
    }
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", fname, "in %.0f s" % secs)


if __name__ == "__main__":
    main()
