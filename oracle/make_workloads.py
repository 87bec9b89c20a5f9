"""Write the synthetic workload table (masses) used by tests and the benchmark.

Run: python -m oracle.make_workloads [names...] [-jN]   (writes synth/workloads.json)

For every workload lattice this generates the gauge field with the seeded
heat-bath, computes m_crit from the spectrum of D(0) with the oracle, and
stores m_crit with the field's plaquette and topological charge, so that a
consumer can regenerate the field and check it is the same one.
Seeds: gauge field rng_for(cfg, round(100 beta), L1, L2, idx).
"""
from __future__ import annotations

import json
import os
import sys
import time

import synth
from oracle import dirac, mg, spectrum

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "synth", "workloads.json")

# (name, cfg, L, beta, idx, sweeps, mass gaps)
WORKLOADS = [
    ("schwinger_32_b6", 1, 32, 6.0, 0, 500, [1e-3]),
    ("schwinger_256_b3", 2, 256, 3.0, 0, 500, [1e-1, 1e-2, 3e-3, 1e-3]),
    ("schwinger_256_b6", 2, 256, 6.0, 0, 500, [1e-1, 1e-2, 3e-3, 1e-3]),
    ("schwinger_256_b10", 2, 256, 10.0, 0, 500, [1e-1, 1e-2, 3e-3, 1e-3]),
    # held-out configurations of the learned setup (same recipe as its training set)
    ("heldout_256_b3", 5, 256, 3.0, 10000, 100, [1e-2, 1e-3]),
    ("heldout_256_b6", 5, 256, 6.0, 10001, 100, [1e-2, 1e-3]),
    ("heldout_256_b10", 5, 256, 10.0, 10002, 100, [1e-2, 1e-3]),
    ("heldout_512_b3", 5, 512, 3.0, 10003, 100, [1e-2, 1e-3]),
    ("heldout_512_b6", 5, 512, 6.0, 10004, 100, [1e-2, 1e-3]),
    ("heldout_512_b10", 5, 512, 10.0, 10005, 100, [1e-2, 1e-3]),
]

def main(names=None, workers=1):
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    todo = [w for w in WORKLOADS if not names or w[0] in names]
    if workers > 1:
        import concurrent.futures as cf
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            done = list(ex.map(entry, todo))
    else:
        done = [entry(w) for w in todo]
    for name, e in done:
        table[name] = e
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("-j")]
    jobs = [int(a[2:]) for a in sys.argv[1:] if a.startswith("-j")]
    main(args or None, jobs[0] if jobs else 1)
