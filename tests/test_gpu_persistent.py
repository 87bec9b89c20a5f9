"""The coarsest-level GCR in one cooperative launch (grid barriers between its
phases) reproduces the oracle's V-cycle: fixed iteration counts with
restarts, the tolerance stop, several right-hand sides, several sites per
wave; in FP32 it agrees with the launch-by-launch sequence."""
import pytest

import synth
from oracle import mg
from gpu_util import dev, host, rel_err, u1_config, vectors

pytestmark = pytest.mark.gpu


def _setup(amg, L, ctol, prec=None):
    U = u1_config(L, L)
    A = mg.wilson_stencil(U, 0.02)
    V1 = (L // 4) ** 2
    vecs = [vectors(4, A.V, 2, 7), vectors(8, V1, 8, 8)]
    kw = dict(blocks=[(4, 4), (2, 2)], nvec=[4, 8], coarse_tol=ctol, coarse_maxiter=12, coarse_restart=5,
              kcycle_tol=0.0, kcycle_maxiter=3, coarse_dense_max=0)
    H = mg.build_hierarchy(A, vecs, mg.MGParams(**kw))
    if prec is not None:
        kw["inner_prec"] = prec
    S = amg.Solver(amg.Gauge(dev(U), 0.02), amg.MGParams(**kw), nullvecs=[dev(v) for v in vecs])
    return A, H, S


@pytest.mark.parametrize("L,nrhs,ctol,blocks", [(32, 1, 0.0, None), (64, 3, 0.0, None), (64, 2, 0.2, None),
                                               (128, 1, 0.0, "8")])
def test_persistent_coarse_solve_matches_oracle_vcycle(monkeypatch, L, nrhs, ctol, blocks):
    import paper_0707_4018_amd as amg
    print(f"persistent coarse solve L={L} nrhs={nrhs} tol={ctol} blocks={blocks}", flush=True)
    monkeypatch.setenv("AMG_PERSISTENT_COARSE", "1")
    if blocks is not None:
        monkeypatch.setenv("AMG_PCOARSE_BLOCKS", blocks)
    A, H, S = _setup(amg, L, ctol)
    b = synth.gaussian_field((nrhs, A.V, 2, 1), synth.rng_for(9, L, nrhs))
    x = host(S.vcycle(dev(b)))
    for i in range(nrhs):
        assert rel_err(x[i].reshape(A.V, 2), mg.vcycle(H, 0, b[i].reshape(A.V, 2))) < 1e-10


def test_persistent_coarse_solve_fp32_matches_launch_sequence(monkeypatch):
    import paper_0707_4018_amd as amg
    print("persistent coarse solve fp32 vs launch sequence", flush=True)
    L, nrhs = 64, 2
    b = synth.gaussian_field((nrhs, L * L, 2, 1), synth.rng_for(10, L))
    monkeypatch.setenv("AMG_PERSISTENT_COARSE", "0")
    _, _, S0 = _setup(amg, L, 0.0, amg.F32)
    x0 = host(S0.vcycle(dev(b)))
    monkeypatch.setenv("AMG_PERSISTENT_COARSE", "1")
    _, _, S1 = _setup(amg, L, 0.0, amg.F32)
    x1 = host(S1.vcycle(dev(b)))
    assert rel_err(x1, x0) < 1e-5
