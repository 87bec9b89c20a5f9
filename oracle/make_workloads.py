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

# four-dimensional SU(3) base configuration: Haar links on 8^3 x 16 smoothed
# by 20 stout steps (rho 0.0215, plaquette about 0.6), tiled periodically to
# the workload volume; (name, dims, seed, rho, steps, mass gaps)
WORKLOADS_4D = [
    ("wilson4d_8x8x8x16", (8, 8, 8, 16), [3, 8, 8, 8, 16], 0.0215, 20, [2e-2]),
]


def su3_base(dims, seed, rho, steps):
    U = synth.su3_haar((4,) + tuple(reversed(dims)), synth.rng_for(*seed))
    return synth.su3_stout_smear(U, rho, steps)


def entry4d(w):
    name, dims, seed, rho, steps, gaps = w
    t0 = time.time()
    U = su3_base(dims, seed, rho, steps)
    A0 = mg.wilson_stencil(U, 0.0)
    mcrit, lam = spectrum.critical_mass(A0)
    e = {"dims": list(dims), "seed": seed, "stout_rho": rho, "stout_steps": steps, "m_crit": mcrit,
         "leftmost_eigenvalue_m0": [lam.real, lam.imag], "mass_gaps": gaps, "masses": [mcrit + g for g in gaps],
         "plaquette": synth.su3_mean_plaquette(U)}
    print(name, e, f"{time.time() - t0:.1f}s", flush=True)
    return name, e


def entry(w):
    name, cfg, L, beta, idx, sweeps, gaps = w
    t0 = time.time()
    seed = [cfg, int(round(100 * beta)), L, L, idx]
    th = synth.u1_heatbath(L, L, beta, sweeps, synth.rng_for(*seed))
    A0 = mg.wilson_stencil(dirac.u1_field(th), 0.0)
    mcrit, lam = spectrum.critical_mass(A0)
    e = {
        "cfg": cfg, "L1": L, "L2": L, "beta": beta, "idx": idx, "sweeps": sweeps,
        "seed": seed, "m_crit": mcrit, "leftmost_eigenvalue_m0": [lam.real, lam.imag],
        "mass_gaps": gaps, "masses": [mcrit + g for g in gaps],
        "plaquette": synth.u1_mean_plaquette(th), "Q": round(synth.u1_topological_charge(th)),
    }
    print(name, e, f"{time.time() - t0:.1f}s", flush=True)
    return name, e


def main(names=None, workers=1):
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    todo = [w for w in WORKLOADS if not names or w[0] in names]
    todo4 = [w for w in WORKLOADS_4D if not names or w[0] in names]
    if workers > 1:
        import concurrent.futures as cf
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            done = list(ex.map(entry, todo)) + list(ex.map(entry4d, todo4))
    else:
        done = [entry(w) for w in todo] + [entry4d(w) for w in todo4]
    for name, e in done:
        table[name] = e
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("-j")]
    jobs = [int(a[2:]) for a in sys.argv[1:] if a.startswith("-j")]
    main(args or None, jobs[0] if jobs else 1)
