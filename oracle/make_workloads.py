"""Write the synthetic workload table (masses) used by tests and the benchmark.

Run: python -m oracle.make_workloads   (writes synth/workloads.json)

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
]


def main(names=None):
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    for name, cfg, L, beta, idx, sweeps, gaps in WORKLOADS:
        if names and name not in names:
            continue
        t0 = time.time()
        seed = [cfg, int(round(100 * beta)), L, L, idx]
        th = synth.u1_heatbath(L, L, beta, sweeps, synth.rng_for(*seed))
        A0 = mg.wilson_stencil(dirac.u1_field(th), 0.0)
        mcrit, lam = spectrum.critical_mass(A0)
        table[name] = {
            "cfg": cfg, "L1": L, "L2": L, "beta": beta, "idx": idx, "sweeps": sweeps,
            "seed": seed, "m_crit": mcrit, "leftmost_eigenvalue_m0": [lam.real, lam.imag],
            "mass_gaps": gaps, "masses": [mcrit + g for g in gaps],
            "plaquette": synth.u1_mean_plaquette(th), "Q": round(synth.u1_topological_charge(th)),
        }
        print(name, table[name], f"{time.time() - t0:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(table, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or None)
