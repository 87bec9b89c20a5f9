"""Write (or check) the synthetic workload table (masses) used by tests and the benchmark.

Run: python -m oracle.make_workloads [names...] [-jN]          (writes synth/workloads.json)
     python -m oracle.make_workloads --check [names...] [-jN]  (recomputes, compares, writes nothing)

Test infrastructure: this script calls only the oracle and the seeded input
generators.  For every workload lattice it generates the gauge field with the
seeded heat-bath, computes m_crit from the spectrum of D(m = 0) with the
oracle (m_crit = -min Re lambda, numerical-test section), and stores m_crit
with the field's plaquette and topological charge, so that a consumer can
regenerate the field and check it is the same one.
Seeds: gauge field rng_for(cfg, round(100 beta), L1, L2, idx).

--check recomputes the listed entries and compares them with the stored
table: plaquette and charge exactly (same seeded generator, same
arithmetic), m_crit to the eigensolver tolerance (CHECK_MCRIT_TOL).
"""
from __future__ import annotations

import json
import os
import sys
import time

import synth
from oracle import dirac, mg, spectrum

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "synth", "workloads.json")

# ARPACK is run to tol 1e-6 on the shift-inverted operator; the eigenvalues
# of D near the shift then carry an absolute error far below this bound.
CHECK_MCRIT_TOL = 1e-8

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


# ensembles of the paper's own test (128^2, beta 6 and 10) in chosen
# topological sectors: the heat-bath starts from the constant flux of charge
# Q (cold for Q = 0) and the first seed index whose field still has charge Q
# is kept (name, L, beta, Q, sweeps, mass gaps)
WORKLOADS_Q = [
    ("paper128_b6_q0", 128, 6.0, 0, 500, [1e-1, 3e-2, 1e-2, 3e-3, 1e-3]),
    ("paper128_b6_q4", 128, 6.0, 4, 500, [1e-1, 3e-2, 1e-2, 3e-3, 1e-3]),
    ("paper128_b10_q0", 128, 10.0, 0, 500, [1e-1, 3e-2, 1e-2, 3e-3, 1e-3]),
    ("paper128_b10_q4", 128, 10.0, 4, 500, [1e-1, 3e-2, 1e-2, 3e-3, 1e-3]),
]


def entry_q(w):
    """(name, entry) of the first seed idx = 0, 1, ... (seed (6, 100 beta, L, L,
    idx)) whose heat-bath field, started from the flux background of charge Q,
    has topological charge Q."""
    name, L, beta, Q, sweeps, gaps = w
    t0 = time.time()
    for idx in range(1000):
        seed = [6, int(round(100 * beta)), L, L, idx]
        th = synth.u1_heatbath(L, L, beta, sweeps, synth.rng_for(*seed), synth.u1_flux(L, L, Q))
        if round(synth.u1_topological_charge(th)) == Q:
            break
    else:
        raise RuntimeError(f"no field with Q = {Q} among 1000 seeds")
    A0 = mg.wilson_stencil(dirac.u1_field(th), 0.0)
    mcrit, lam = spectrum.critical_mass(A0)
    e = {
        "cfg": 6, "L1": L, "L2": L, "beta": beta, "idx": idx, "sweeps": sweeps, "start_flux_Q": Q,
        "seed": seed, "m_crit": mcrit, "leftmost_eigenvalue_m0": [lam.real, lam.imag],
        "mass_gaps": gaps, "masses": [mcrit + g for g in gaps],
        "plaquette": synth.u1_mean_plaquette(th), "Q": round(synth.u1_topological_charge(th)),
    }
    print(name, f"idx {idx} m_crit {mcrit:.12f} Q {e['Q']} ({time.time() - t0:.1f} s)", flush=True)
    return name, e


def entry(w):
    """(name, table entry) of one 2d U(1) workload."""
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
    print(name, f"m_crit {mcrit:.12f} plaquette {e['plaquette']!r} Q {e['Q']} ({time.time() - t0:.1f} s)",
          flush=True)
    return name, e


def compare(stored: dict, new: dict) -> list[str]:
    """Differences between a stored entry and a recomputed one (empty: identical)."""
    bad = []
    for k in ("cfg", "L1", "L2", "beta", "idx", "sweeps", "seed", "mass_gaps", "Q"):
        if stored.get(k) != new[k]:
            bad.append(f"{k}: stored {stored.get(k)!r} new {new[k]!r}")
    if stored.get("plaquette") != new["plaquette"]:
        bad.append(f"plaquette: stored {stored.get('plaquette')!r} new {new['plaquette']!r}")
    dm = abs(stored["m_crit"] - new["m_crit"])
    if not dm <= CHECK_MCRIT_TOL:
        bad.append(f"m_crit: stored {stored['m_crit']!r} new {new['m_crit']!r} (|diff| {dm:.2e})")
    for a, b in zip(stored["masses"], new["masses"]):
        if not abs(a - b) <= CHECK_MCRIT_TOL:
            bad.append(f"mass: stored {a!r} new {b!r}")
    return bad


def _one(w):
    return entry_q(w) if len(w) == 6 else entry(w)


def _run(todo, workers):
    if workers > 1:
        import concurrent.futures as cf
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_one, todo))
    return [_one(w) for w in todo]


def main(names=None, workers=1, check=False) -> int:
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    todo = [w for w in WORKLOADS + WORKLOADS_Q if not names or w[0] in names]
    done = _run(todo, workers)
    if check:
        nbad = 0
        for name, e in done:
            bad = compare(table[name], e) if name in table else ["not in the stored table"]
            print(f"{name}: {'identical' if not bad else 'DIFFERS'}"
                  f" (|dm_crit| {abs(table.get(name, e)['m_crit'] - e['m_crit']):.2e})", flush=True)
            for b in bad:
                print("   ", b)
            nbad += bool(bad)
        return 1 if nbad else 0
    for name, e in done:
        table[name] = e
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1)
    return 0


if __name__ == "__main__":
    argv = sys.argv[1:]
    check = "--check" in argv
    args = [a for a in argv if not a.startswith("-")]
    jobs = [int(a[2:]) for a in argv if a.startswith("-j")]
    sys.exit(main(args or None, jobs[0] if jobs else 1, check))
