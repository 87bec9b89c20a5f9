"""Helpers shared by the GPU tests: move seeded inputs to the device, compare."""
import numpy as np

import synth
from oracle import dirac


def dev(a: np.ndarray, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b|| / ||b||."""
    nb = np.linalg.norm(np.ravel(b))
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0))


def max_rel_err(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| (element by element)."""
    return float(np.abs(np.ravel(a) - np.ravel(b)).max() / max(np.abs(np.ravel(b)).max(), 1e-300))


def u1_config(L1, L2, beta=6.0, sweeps=40, seed=0):
    th = synth.u1_heatbath(L1, L2, beta, sweeps, synth.rng_for(90, int(100 * beta), L1, L2, seed))
    return dirac.u1_field(th)          # (2, L2, L1, 1, 1)


def su3_config(dims, seed=0, smear=0):
    U = synth.su3_haar((4,) + tuple(reversed(dims)), synth.rng_for(91, *dims, seed))
    if smear:
        U = synth.su3_stout_smear(U, 0.1, smear)
    return U


def vectors(n, V, dof, seed):
    return np.stack([synth.gaussian_field((V, dof), synth.rng_for(92, seed, k)) for k in range(n)])
