#!/usr/bin/env python3
"""Train the near-null-vector proposal network on the GPU and evaluate the learned setup.

Data (seeded, synthetic): U(1) heat-bath configurations on L x L lattices
(cold start, `sweeps` checkerboard sweeps of the Wilson plaquette action),
beta cycling through {3, 6, 10} with the configuration index, seeds
[5, round(100 beta), L, L, idx]; training indices 0..n-1, held-out indices
from 10000.  Targets: the level-0 near-null vectors of the library's adaptive
setup (4x4 blocks, 8 vectors, nu0 MR steps on the first vector, ncyc
error-propagation sweeps per further vector; defaults 20 and 2) at mass m_crit(beta) + 0.01, m_crit interpolated in 1/beta from
the workload table.

Usage:
  python -m paper_0707_4018_amd.train_cnn --n 2000 --L 128 --epochs 30 --out weights.npz
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

BETAS = (3.0, 6.0, 10.0)
HELD_OUT = 10000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def m_crit(beta: float) -> float:
    """Critical mass interpolated linearly in 1/beta between the tabulated ensembles."""
    w = json.load(open(os.path.join(ROOT, "synth", "workloads.json")))
    bs = np.array(BETAS)
    mc = np.array([w[f"schwinger_256_b{int(b)}"]["m_crit"] for b in BETAS])
    return float(np.interp(1.0 / beta, (1.0 / bs)[::-1], mc[::-1]))


def config(args):
    """(idx, theta) of configuration idx (worker process, no GPU)."""
    idx, L, sweeps = args
    beta = BETAS[idx % 3]
    th = synth.u1_heatbath(L, L, beta, sweeps, synth.rng_for(5, int(round(100 * beta)), L, L, idx))
    return idx, th


def ensemble(indices, L, sweeps, workers=16):
    out = {}
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for n, (i, th) in enumerate(ex.map(config, [(i, L, sweeps) for i in indices], chunksize=4), 1):
            out[i] = th
            if n % 200 == 0:
                log(f"heat bath: {n}/{len(indices)} configurations")
    return [out[i] for i in indices]


def init_vectors(idx, L, nvecs=(8,), blocks=((4, 4),)):
    """Random starting vectors of the adaptive setup, one set per coarsening."""
    out = []
    V, dof = L * L, 2
    Lc = L
    for l, nv in enumerate(nvecs):
        out.append(np.stack([synth.gaussian_field((V, dof), synth.rng_for(5, 1, idx, l, k)) for k in range(nv)]))
        Lc //= blocks[l][0]
        V, dof = Lc * Lc, 2 * nv
    return out


def target_params(amg):
    return amg.MGParams(blocks=[(4, 4)], nvec=[8], coarse_tol=0.1, coarse_maxiter=100, coarse_restart=16)


def build_data(amg, torch, indices, L, sweeps, ths=None, nu0=20, ncyc=2):
    from paper_0707_4018_amd import learned
    if ths is None:
        ths = ensemble(indices, L, sweeps)
    links, targets = [], []
    p = target_params(amg)
    t0 = time.perf_counter()
    for idx, th in zip(indices, ths):
        U = torch.from_numpy(np.exp(1j * th).reshape(2, L * L)).cuda()
        init = [torch.from_numpy(v).cuda() for v in init_vectors(idx, L)]
        targets.append(learned.adaptive_targets(U, L, L, m_crit(BETAS[idx % 3]) + 0.01, p, init, nu0=nu0, ncyc=ncyc))
        links.append(U)
        if len(links) % 200 == 0:
            log(f"targets: {len(links)}/{len(indices)}")
    torch.cuda.synchronize()
    log(f"targets for {len(indices)} configurations: {time.perf_counter() - t0:.1f} s")
    return torch.stack(links), torch.stack(targets)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--n-val", type=int, default=48)
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-final", type=float, default=3e-4)
    ap.add_argument("--fp32", action="store_true", help="FP32 activations instead of bfloat16")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--target-nu0", type=int, default=20, help="MR steps on the first adaptive vector")
    ap.add_argument("--target-ncyc", type=int, default=2, help="error-propagation sweeps per further vector")
    ap.add_argument("--out", default="cnn_weights.npz")
    args = ap.parse_args(argv)

    train_idx = list(range(args.n))
    val_idx = list(range(HELD_OUT, HELD_OUT + args.n_val))
    t0 = time.perf_counter()
    ths = ensemble(train_idx + val_idx, args.L, args.sweeps)
    log(f"heat bath: {len(ths)} configurations {args.L}^2 x {args.sweeps} sweeps in {time.perf_counter() - t0:.1f} s")

    import torch
    import paper_0707_4018_amd as amg
    from paper_0707_4018_amd import learned

    Lt = args.L
    tk = dict(nu0=args.target_nu0, ncyc=args.target_ncyc)
    links, targets = build_data(amg, torch, train_idx, Lt, args.sweeps, ths[:args.n], **tk)
    vlinks, vtargets = build_data(amg, torch, val_idx, Lt, args.sweeps, ths[args.n:], **tk)
    net = amg.Cnn(learned.init_params(args.seed), bf16=not args.fp32)
    v0 = learned.evaluate_loss(net, vlinks, vtargets, Lt, Lt)
    t0 = time.perf_counter()
    hist = learned.train(net, links, targets, Lt, Lt, args.epochs, args.batch, args.lr, seed=args.seed,
                         lr_final=args.lr_final, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    v1 = learned.evaluate_loss(net, vlinks, vtargets, Lt, Lt)
    log(f"validation loss {v0:.4f} -> {v1:.4f}; training {t_train:.1f} s")
    learned.save(args.out, net, train_loss=np.array(hist), val_loss_init=v0, val_loss=v1, n_train=args.n,
                 L=Lt, sweeps=args.sweeps, epochs=args.epochs, batch=args.batch, bf16=int(not args.fp32),
                 train_seconds=t_train, target_nu0=args.target_nu0, target_ncyc=args.target_ncyc)
    print(json.dumps({"n_train": args.n, "L": Lt, "epochs": args.epochs, "val_loss_init": v0, "val_loss": v1,
                      "train_loss": hist, "train_seconds": t_train}))


if __name__ == "__main__":
    main()
