"""Batched solves (one launch per stage over many instances, hipGraph replay):
each instance must reach the true FP64 residual 1e-10 under the oracle's D and
agree with its own single-instance solve; uneven lattices and rhs counts."""
import numpy as np
import pytest

import synth
from oracle import mg
from gpu_util import dev, host, rel_err, u1_config, vectors

pytestmark = pytest.mark.gpu


def _instances(sizes, nrhs, mixed, seed=0):
    import paper_0707_4018_amd as amg
    out = []
    for i, (L, nr) in enumerate(zip(sizes, nrhs)):
        U = u1_config(L, L, beta=3.0 + i, sweeps=30, seed=seed + i)
        m = 0.02 + 0.01 * i
        A = mg.wilson_stencil(U, m)
        # coarsest level by GCR (what batched solves run) also in the single solves compared with
        p = amg.MGParams(blocks=[(4, 4), (2, 2)], nvec=[4, 4], coarse_tol=0.1, coarse_maxiter=40,
                         kcycle_tol=0.1, kcycle_maxiter=4, inner_prec=amg.F32 if mixed else amg.F64, p_bf16=mixed,
                         coarse_dense_max=0)
        g = amg.Gauge(dev(U), m)
        V1 = (L // 4) ** 2
        init = [vectors(4, L * L, 2, 100 + i), vectors(4, V1, 8, 200 + i)]
        S = amg.Solver(g, p, init=[dev(v) for v in init])
        b = synth.gaussian_field((nr, L * L, 2, 1), synth.rng_for(300, i))
        out.append((A, g, S, b))
    return out


@pytest.mark.parametrize("mixed", [False, True])
def test_batch_matches_single_solves(mixed):
    import paper_0707_4018_amd as amg
    sizes, nrhs = [16, 32, 24, 48], [1, 3, 2, 1]
    print(f"batch sizes {sizes} nrhs {nrhs} mixed {mixed}", flush=True)
    inst = _instances(sizes, nrhs, mixed)
    B = amg.Batch([s for _, _, s, _ in inst], nrhs, autotune=True)
    info = B.info()
    assert info["red_block_cap"] in (128, 256, 512, 1024) and info["launches_per_outer_step"] > 10
    # the joint search: 4 reduction grids x 2 coarse stencils, the fastest kept
    tr = info["tuning"]
    assert len(tr) == 8 and {(t["red_block_cap"], t["coarse_mrhs_mfma"]) for t in tr} == {
        (c, m) for c in (128, 256, 512, 1024) for m in (True, False)}
    best = min(tr, key=lambda t: t["ms_per_outer_step"])
    assert (best["red_block_cap"], best["coarse_mrhs_mfma"]) == (info["red_block_cap"], info["coarse_mrhs_mfma"])
    psis, infos = B.solve([dev(b) for _, _, _, b in inst], tol=1e-10)
    q = 0
    for (A, g, S, b), psi in zip(inst, psis):
        psi = host(psi)
        single, _ = S.solve(dev(b), tol=1e-10)
        single = host(single)
        for j in range(b.shape[0]):
            res = mg.norm(b[j].reshape(A.V, 2) - A.apply(psi[j].reshape(A.V, 2))) / mg.norm(b[j])
            assert infos[q].converged and res <= 1e-10, (q, res)
            assert rel_err(psi[j], single[j]) < 1e-7
            q += 1
    # a second solve through the same graphs (replays are reusable)
    psis2, infos2 = B.solve([dev(b) for _, _, _, b in inst], tol=1e-10)
    for p1, p2 in zip(psis, psis2):
        assert rel_err(host(p2), host(p1)) < 1e-9


@pytest.mark.parametrize("mrhs", ["0", "1"])
def test_batch_coarse_stencil_choices_agree(mrhs, monkeypatch):
    """Both coarse-stencil choices the tuner picks between give the single
    solves' answers (no autotune; the choice set through the environment)."""
    import paper_0707_4018_amd as amg
    monkeypatch.setenv("AMG_BATCH_MRHS", mrhs)
    sizes, nrhs = [16, 32], [2, 1]
    print(f"batch coarse stencil mrhs={mrhs}", flush=True)
    inst = _instances(sizes, nrhs, True)
    B = amg.Batch([s for _, _, s, _ in inst], nrhs, autotune=False)
    assert B.info()["coarse_mrhs_mfma"] == (mrhs == "1") and B.info()["tuning"] == []
    psis, infos = B.solve([dev(b) for _, _, _, b in inst], tol=1e-10)
    for (A, g, S, b), psi in zip(inst, psis):
        single, _ = S.solve(dev(b), tol=1e-10)
        assert rel_err(host(psi), host(single)) < 1e-7
    assert all(i.converged for i in infos)


def test_batch_rejects_mismatched_solvers():
    import paper_0707_4018_amd as amg
    inst = _instances([16], [1], False)
    U = u1_config(16, 16)
    g = amg.Gauge(dev(U), 0.1)
    p = amg.MGParams(blocks=[(4, 4)], nvec=[4])
    S2 = amg.Solver(g, p, init=[dev(vectors(4, 256, 2, 5))])
    with pytest.raises(amg.AMGError):
        amg.Batch([inst[0][2], S2], [1, 1])


def test_fused_gcr_step_matches_oracle_vcycle(monkeypatch):
    """The opt-in two-launch GCR step on 16-dof levels gives the same V-cycle as the oracle."""
    import paper_0707_4018_amd as amg
    monkeypatch.setenv("AMG_FUSED_GCR", "1")
    U = u1_config(32, 32)
    A = mg.wilson_stencil(U, 0.02)
    vecs = [vectors(4, A.V, 2, 7), vectors(8, 64, 8, 8)]
    po = mg.MGParams(blocks=[(4, 4), (2, 2)], nvec=[4, 8], coarse_tol=0.0, coarse_maxiter=12, coarse_restart=5,
                     kcycle_tol=0.0, kcycle_maxiter=3, coarse_dense_max=0)
    H = mg.build_hierarchy(A, vecs, po)
    pg = amg.MGParams(blocks=[(4, 4), (2, 2)], nvec=[4, 8], coarse_tol=0.0, coarse_maxiter=12, coarse_restart=5,
                      kcycle_tol=0.0, kcycle_maxiter=3, coarse_dense_max=0)
    S = amg.Solver(amg.Gauge(dev(U), 0.02), pg, nullvecs=[dev(v) for v in vecs])
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(9))
    x = host(S.vcycle(dev(b)))[0].reshape(A.V, 2)
    assert rel_err(x, mg.vcycle(H, 0, b[0].reshape(A.V, 2))) < 1e-10
