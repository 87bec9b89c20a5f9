"""The exact coarsest solve (dense inverse by Gauss-Jordan on the GPU) against
the oracle, whose coarsest solve is an LU solve of the same Galerkin matrix.

A V-cycle whose coarsest level is solved exactly satisfies the Galerkin
property: without post-smoothing the residual after the coarse-grid
correction is orthogonal to the range of P (P^dag r = 0).  That is checked
with the oracle's operator and prolongator, independently of the oracle's
V-cycle, and the GPU V-cycle is compared with the oracle's element by
element.  Coarsest levels of 96 to 4096 unknowns (ragged against the 64 x 64
tiles of the elimination), FP64 and the FP32 copy of the inverse, and the
refresh of the inverse after a mass change.
"""
import numpy as np
import pytest

import synth
from oracle import mg
from gpu_util import dev, host, max_rel_err, rel_err, u1_config, vectors

pytestmark = pytest.mark.gpu


def _given(L1, L2, block, nv, m=0.05, seed=0, **kw):
    import paper_0707_4018_amd as amg
    U = u1_config(L1, L2, seed=seed)
    A = mg.wilson_stencil(U, m)
    po = mg.MGParams(blocks=[block], nvec=[nv], **kw)
    pg = amg.MGParams(blocks=[block], nvec=[nv], **kw)
    vecs = [vectors(nv, A.V, 2, seed + 40)]
    H = mg.build_hierarchy(A, vecs, po)
    S = amg.Solver(amg.Gauge(dev(U), m), pg, nullvecs=[dev(v) for v in vecs])
    return U, A, H, S, vecs


# (L1, L2, block, nv): coarsest unknowns 96, 120, 768, 1024, 4096
CASES = [(8, 8, (2, 2), 3), (12, 8, (2, 4), 5), (32, 32, (4, 4), 6), (32, 32, (4, 4), 8), (64, 64, (4, 4), 8)]


@pytest.mark.parametrize("L1,L2,block,nv", CASES)
def test_exact_coarsest_vcycle_matches_oracle(L1, L2, block, nv):
    print(f"dense coarsest {L1}x{L2} block {block} nv {nv}", flush=True)
    U, A, H, S, _ = _given(L1, L2, block, nv)
    N = H.ops[1].V * H.ops[1].dof
    assert N <= 4096
    b = synth.gaussian_field((2, A.V, 2, 1), synth.rng_for(50, L1, L2))
    x = host(S.vcycle(dev(b)))
    for k in range(2):
        xo = mg.vcycle(H, 0, b[k].reshape(A.V, 2))
        assert max_rel_err(x[k].reshape(A.V, 2), xo) < 1e-10, k


@pytest.mark.parametrize("L1,L2,block,nv", [CASES[1], CASES[3], CASES[4]])
def test_exact_coarse_correction_is_galerkin_orthogonal(L1, L2, block, nv):
    """nu_post = 0: P^dag (b - D x) = 0 after the V-cycle, with the oracle's D and P."""
    print(f"galerkin orthogonality {L1}x{L2}", flush=True)
    U, A, H, S, _ = _given(L1, L2, block, nv, nu_post=0)
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(51, L1, L2))
    x = host(S.vcycle(dev(b)))[0].reshape(A.V, 2)
    r = b[0].reshape(A.V, 2) - A.apply(x)
    assert mg.norm(H.Ps[0].restrict(r)) < 1e-11 * mg.norm(b)
    assert mg.norm(r) > 1e-3 * mg.norm(b)      # the residual itself is not zero


def test_exact_coarsest_fp32_copy():
    """FP32 cycle with the FP32 copy of the inverse against the FP64 oracle cycle."""
    import torch
    import paper_0707_4018_amd as amg
    print("dense coarsest fp32", flush=True)
    U, A, H, S, vecs = _given(32, 32, (4, 4), 8)
    pg = amg.MGParams(blocks=[(4, 4)], nvec=[8], inner_prec=amg.F32)
    S32 = amg.Solver(amg.Gauge(dev(U), 0.05), pg, nullvecs=[dev(v) for v in vecs])
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(52))
    x = host(S32.vcycle(dev(b)))[0].reshape(A.V, 2)
    assert rel_err(x, mg.vcycle(H, 0, b[0].reshape(A.V, 2))) < 1e-4


def test_exact_coarsest_after_mass_change():
    """set_mass shifts every coarse operator and refreshes the inverse."""
    import paper_0707_4018_amd as amg
    print("dense coarsest after set_mass", flush=True)
    U, A, H, S, vecs = _given(16, 16, (4, 4), 4)
    S.set_mass(0.2)
    H2 = mg.build_hierarchy(mg.wilson_stencil(U, 0.2), vecs, mg.MGParams(blocks=[(4, 4)], nvec=[4]))
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(53))
    x = host(S.vcycle(dev(b)))[0].reshape(A.V, 2)
    assert max_rel_err(x, mg.vcycle(H2, 0, b[0].reshape(A.V, 2))) < 1e-10


def test_exact_coarsest_solve_converges_like_oracle():
    """FGCR with the exact coarsest solve: true residual 1e-10 with the oracle's D,
    iteration count equal to the oracle's within one."""
    print("dense coarsest solve", flush=True)
    U, A, H, S, _ = _given(32, 32, (4, 4), 8, m=0.02)
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(54))
    psi, info = S.solve(dev(b), tol=1e-10)
    psi = host(psi)[0].reshape(A.V, 2)
    res = mg.norm(b[0].reshape(A.V, 2) - A.apply(psi)) / mg.norm(b)
    assert info[0].converged and res <= 1e-10
    _, io = mg.mg_solve(H, b[0].reshape(A.V, 2), 1e-10)
    assert abs(info[0].iters - io.iters) <= 1, (info[0].iters, io.iters)
