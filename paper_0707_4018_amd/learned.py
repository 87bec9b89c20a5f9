"""Learned setup: training and use of the near-null-vector proposal network.

Host-side sequencing only.  Targets are the level-0 near-null vectors that
the library's own adaptive setup produces (Eq. (4) and the adaptive procedure
after Eq. (5)); every training step (forward, projection loss, backward,
Adam) and every proposal runs in libamg's kernels.  This module draws
minibatches, calls those entry points, and saves/loads the flat parameter
vector (.npz, numpy arrays only).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .binding import Cnn, Gauge, MGParams, Solver

CHANNELS = Cnn.CHANNELS


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation: W ~ N(0, 1/(9 c_in)), b = 0, flat float32 in ABI order."""
    rng = np.random.default_rng([5150, seed])
    parts = []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        parts.append((rng.standard_normal((co, ci, 3, 3)) * np.sqrt(1.0 / (9 * ci))).ravel())
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def save(path: str, net: Cnn, **meta):
    np.savez(path, params=net.params(), **{k: np.asarray(v) for k, v in meta.items()})


def load(path: str, bf16: bool = True) -> Cnn:
    with np.load(path, allow_pickle=False) as z:
        return Cnn(z["params"], bf16=bf16)


def adaptive_targets(links: torch.Tensor, L1: int, L2: int, mass: float, params: MGParams, init: list,
                     nu0: int = 20, ncyc: int = 2) -> torch.Tensor:
    """Level-0 near-null vectors (8, V, 2) of the adaptive setup for one configuration.

    links: (2, L1 * L2) complex128 on the GPU (canonical U(1) layout)."""
    g = Gauge(links.reshape(2, L2, L1, 1, 1), mass)
    S = Solver(g, params, init=init, nu0=nu0, ncyc=ncyc)
    v = S.nullvecs(0)
    del S, g
    return v


def train(net: Cnn, links: torch.Tensor, targets: torch.Tensor, L1: int, L2: int, epochs: int, batch: int,
          lr: float, seed: int = 0, lr_final: float | None = None, log=None):
    """Adam over shuffled minibatches of `batch` configurations.

    links (N, 2, V), targets (N, 8, V, 2) complex128 on the GPU.  The learning
    rate decays geometrically from lr to lr_final over all steps.  Returns
    the per-epoch mean training loss."""
    n = links.shape[0]
    rng = np.random.default_rng([6060, seed])
    steps = epochs * max(1, n // batch)
    decay = 1.0 if lr_final is None else (lr_final / lr) ** (1.0 / max(1, steps - 1))
    hist = []
    k = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot, cnt = 0.0, 0
        t0 = time.perf_counter()
        for i in range(0, n - batch + 1, batch):
            idx = torch.from_numpy(np.sort(perm[i:i + batch])).to(links.device)
            tot += net.train_step(links.index_select(0, idx), targets.index_select(0, idx), L1, L2,
                                  lr * decay ** k)
            cnt += 1
            k += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f} ({time.perf_counter() - t0:.2f} s)")
    return hist


def evaluate_loss(net: Cnn, links: torch.Tensor, targets: torch.Tensor, L1: int, L2: int, batch: int = 8) -> float:
    """Mean projection loss of the network's proposals on held-out data."""
    n = links.shape[0]
    tot = 0.0
    for i in range(0, n, batch):
        j = min(n, i + batch)
        tot += net.loss_grad(links[i:j], targets[i:j], L1, L2, grads=False)[0] * (j - i)
    return tot / n
