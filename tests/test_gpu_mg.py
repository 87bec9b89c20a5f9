"""Parity of the multigrid pieces (HIP, through the C ABI) with the oracle.

Same seeded inputs on both sides (the near-null vectors or the adaptive
setup's random starting vectors are passed to both).  FP64 pieces must agree
to ~1e-12 (single operations) or ~1e-10 (a V-cycle, which chains dozens of
reductions); every solve must reach the true FP64 relative residual 1e-10,
recomputed here with the oracle's D.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import dirac, mg
from gpu_util import dev, host, max_rel_err, rel_err, u1_config, vectors, su3_config

pytestmark = pytest.mark.gpu


def _params(blocks, nvec, **kw):
    import paper_0707_4018_amd as amg
    o = mg.MGParams(blocks=list(blocks), nvec=list(nvec))
    g = amg.MGParams(blocks=list(blocks), nvec=list(nvec))
    for k, v in kw.items():
        setattr(o, k, v)
        setattr(g, k, v)
    if o.kcycle_tol is None:          # plain V-cycle on both sides
        g.kcycle_tol, g.kcycle_maxiter = 0.1, 0
    return o, g


def _given(L1, L2, blocks, nvec, m=0.05, seed=0, **kw):
    """Oracle hierarchy and GPU solver built from the same random vectors."""
    import paper_0707_4018_amd as amg
    U = u1_config(L1, L2, seed=seed)
    A = mg.wilson_stencil(U, m)
    po, pg = _params(blocks, nvec, **kw)
    vecs = []
    V, dof, dims = A.V, 2, (L1, L2)
    for l, (b, nv) in enumerate(zip(blocks, nvec)):
        vecs.append(vectors(nv, V, dof, seed * 10 + l))
        dims = tuple(d // bb for d, bb in zip(dims, b))
        V, dof = int(np.prod(dims)), 2 * nv
    H = mg.build_hierarchy(A, vecs, po)
    g = amg.Gauge(dev(U), m)
    S = amg.Solver(g, pg, nullvecs=[dev(v) for v in vecs])
    return U, A, H, g, S


@pytest.mark.parametrize("L1,L2,block,nv", [(32, 32, (4, 4), 8), (8, 8, (4, 4), 4), (4, 4, (4, 4), 3),
                                           (16, 8, (4, 2), 2), (12, 8, (2, 4), 5)])
def test_coarse_operator_matches_oracle(L1, L2, block, nv):
    print(f"galerkin {L1}x{L2} block {block} nv {nv}", flush=True)
    U, A, H, g, S = _given(L1, L2, [block], [nv])
    Y = host(S.coarse_op(1))
    Ac = H.ops[1]
    assert max_rel_err(Y[:, 0], Ac.diag) < 1e-12
    for d in range(4):
        assert max_rel_err(Y[:, 1 + d], Ac.hop[d]) < 1e-12


def test_three_level_operator_and_transfers():
    print("three-level 32x32 (4,4)+(2,2)", flush=True)
    U, A, H, g, S = _given(32, 32, [(4, 4), (2, 2)], [4, 3])
    Y2 = host(S.coarse_op(2))
    assert max_rel_err(Y2[:, 0], H.ops[2].diag) < 1e-11
    for d in range(4):
        assert max_rel_err(Y2[:, 1 + d], H.ops[2].hop[d]) < 1e-11
    for lvl in range(2):
        P = H.Ps[lvl]
        r = synth.gaussian_field((1, H.ops[lvl].V, H.ops[lvl].dof), synth.rng_for(5, lvl))
        e = synth.gaussian_field((1, P.Vc, P.nc), synth.rng_for(6, lvl))
        assert max_rel_err(host(S.restrict(lvl, dev(r)))[0], P.restrict(r[0])) < 1e-12
        assert max_rel_err(host(S.prolong(lvl, dev(e)))[0], P.prolong(e[0])) < 1e-12


def test_coarse_apply_and_mr_match_oracle():
    import paper_0707_4018_amd as amg
    import torch
    U, A, H, g, S = _given(32, 16, [(4, 4)], [8])
    Ac = H.ops[1]
    e = synth.gaussian_field((1, Ac.V, Ac.dof), synth.rng_for(7))
    assert max_rel_err(host(S.level_apply(1, dev(e)))[0], Ac.apply(e[0])) < 1e-12
    assert max_rel_err(host(S.level_apply(1, dev(e), dagger=True))[0], Ac.apply_dagger(e[0])) < 1e-12
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(8))
    x = host(S.mr(0, 3, dev(b)))
    xo = mg.mr(A, b[0].reshape(A.V, 2), 3, 0.8)[0]
    assert max_rel_err(x.reshape(-1), xo.reshape(-1)) < 1e-12
    xc = host(S.mr(1, 2, dev(e)))
    xco = mg.mr(Ac, e[0], 2, 0.8)[0]
    assert max_rel_err(xc.reshape(-1), xco.reshape(-1)) < 1e-12
    # FP32 coarse operator (rounded from the FP64 Galerkin product)
    _, pg = _params([(4, 4)], [8], inner_prec=amg.F32)
    S32 = amg.Solver(g, pg, nullvecs=S._keep)
    out = host(S32.level_apply(1, dev(e, torch.complex64), prec=amg.F32))[0]
    assert rel_err(out, Ac.apply(e[0])) < 1e-5


@pytest.mark.parametrize("dense", [4096, 0])
@pytest.mark.parametrize("blocks,nvec,kc", [([(4, 4)], [6], 0), ([(4, 4), (2, 2)], [4, 4], 0),
                                            ([(4, 4), (2, 2)], [4, 4], 3), ([(4, 4)], [8], 0),
                                            ([(4, 4), (2, 2)], [4, 8], 3)])
def test_vcycle_matches_oracle(blocks, nvec, kc, dense):
    """dense = 4096: the coarsest level is solved exactly (dense inverse);
    dense = 0: by GCR (12 steps, restart 5) on both sides."""
    print(f"vcycle {blocks} {nvec} kcycle {kc} dense {dense}", flush=True)
    U, A, H, g, S = _given(32, 32, blocks, nvec, m=0.02, coarse_tol=0.0, coarse_maxiter=12, coarse_restart=5,
                           kcycle_tol=0.0 if kc else None, kcycle_maxiter=kc if kc else 8, coarse_dense_max=dense)
    assert (S.params.kcycle_maxiter > 0) == bool(kc)
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(9))
    x = host(S.vcycle(dev(b)))[0].reshape(A.V, 2)
    xo = mg.vcycle(H, 0, b[0].reshape(A.V, 2))
    assert rel_err(x, xo) < 1e-10


@pytest.mark.parametrize("eo", [False, True])
@pytest.mark.parametrize("blocks,nvec,kc", [([(4, 4)], [6], 0), ([(4, 4), (2, 2)], [4, 4], 3),
                                            ([(4, 4), (2, 2)], [4, 8], 0)])
def test_vcycle_block_jacobi_matches_oracle(blocks, nvec, kc, eo):
    """The coarsest GCR right-preconditioned by the inverse diagonal blocks
    (12 steps, restart 5, no dense solve) on both sides: the HIP path runs GCR
    on the stencil of A M and returns M y.  Again after a mass change, which
    rebuilds the block inverses and that stencil.  eo: GCR on the even sites
    of the reduced system (two half-lattice launches per step), then the odd
    sites and M y.  (On the 4^2 coarsest levels of the three-level cases 12
    steps solve to rounding with or without the preconditioner; the two-level
    case's 8^2 x 12 level shows that it acts.)"""
    print(f"vcycle block-jacobi {blocks} {nvec} kcycle {kc} eo {eo}", flush=True)
    kw = dict(coarse_tol=0.0, coarse_maxiter=12, coarse_restart=5, kcycle_tol=0.0 if kc else None,
              kcycle_maxiter=kc if kc else 8, coarse_dense_max=0)
    U, A, H, g, S = _given(32, 32, blocks, nvec, m=0.02, coarse_jacobi=True, coarse_eo=eo, **kw)
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(9))
    x = host(S.vcycle(dev(b)))[0].reshape(A.V, 2)
    xo = mg.vcycle(H, 0, b[0].reshape(A.V, 2))
    assert rel_err(x, xo) < 1e-10
    if len(blocks) == 1:                           # the unpreconditioned cycle is another operator
        po, _ = _params(blocks, nvec, **kw)
        Hp = mg.Hierarchy(H.ops, H.Ps, po, H.mass_mats)
        assert rel_err(x, mg.vcycle(Hp, 0, b[0].reshape(A.V, 2))) > 1e-6
    S.set_mass(0.06)
    x2 = host(S.vcycle(dev(b)))[0].reshape(A.V, 2)
    assert rel_err(x2, mg.vcycle(mg.with_mass(H, 0.04), 0, b[0].reshape(A.V, 2))) < 1e-10


def test_mixed_solve_block_jacobi_near_critical():
    """Three-level mixed-precision solve near the critical mass with the
    block-Jacobi coarsest GCR, with and without the even-odd reduction: true
    FP64 residual 1e-10, iteration count within two of the oracle's with the
    same coarsest solver, and fewer coarse operator applications (a reduced
    Schur product counted as one) than without each."""
    import paper_0707_4018_amd as amg
    print("mixed solve with block-jacobi coarsest GCR, 32^2", flush=True)
    L = 32
    U = u1_config(L, L, beta=6.0, sweeps=100, seed=8)
    m = _mcrit(U) + 0.003
    A = mg.wilson_stencil(U, m)
    kw = dict(coarse_tol=0.2, coarse_maxiter=100, coarse_restart=10, kcycle_tol=0.2, kcycle_maxiter=8,
              coarse_dense_max=0)
    init = [vectors(8, A.V, 2, 81), vectors(8, (L // 4) ** 2, 16, 82)]
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(83))
    res = {}
    for jac, eo in ((False, False), (True, False), (True, True)):
        po, pg = _params([(4, 4), (2, 2)], [8, 8], coarse_jacobi=jac, coarse_eo=eo, **kw)
        pg.inner_prec, pg.p_bf16 = amg.F32, True
        S = amg.Solver(amg.Gauge(dev(U), m), pg, init=[dev(v) for v in init], nu0=20, ncyc=4)
        psi, info = S.solve(dev(b), tol=1e-10)
        r = mg.norm(b[0].reshape(A.V, 2) - A.apply(host(psi)[0].reshape(A.V, 2))) / mg.norm(b)
        assert info[0].converged and r <= 1e-10, (jac, eo, r)
        res[jac, eo] = info[0]
        if jac:
            Ho, _ = mg.adaptive_setup(A, po, init, nu0=20, ncyc=4)
            _, io = mg.mg_solve(Ho, b[0].reshape(A.V, 2), 1e-10, 200)
            assert abs(info[0].iters - io.iters) <= 2, (eo, info[0].iters, io.iters)
    n = {k: v.n_coarse for k, v in res.items()}
    assert n[True, False] < n[False, False] and n[True, True] < n[True, False], n


def _mcrit(U):
    ev = np.linalg.eigvals(dirac.dense_D(U, 0.0))
    return -ev.real.min()


def test_adaptive_setup_and_solve_fp64():
    import paper_0707_4018_amd as amg
    L = 32
    U = u1_config(L, L, beta=6.0, sweeps=100, seed=3)
    m = _mcrit(U) + 0.01
    A = mg.wilson_stencil(U, m)
    po, pg = _params([(4, 4)], [8], coarse_tol=0.05, coarse_maxiter=200, coarse_restart=16)
    init = [vectors(8, A.V, 2, 33)]
    Ho, vo = mg.adaptive_setup(A, po, init)
    g = amg.Gauge(dev(U), m)
    S = amg.Solver(g, pg, init=[dev(v) for v in init])
    v = host(S.nullvecs(0))
    assert rel_err(v, vo[0]) < 1e-6
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(0))
    psi, info = S.solve(dev(b), tol=1e-10)
    psi = host(psi)[0].reshape(A.V, 2)
    res = mg.norm(b[0].reshape(A.V, 2) - A.apply(psi)) / mg.norm(b)
    assert info[0].converged and res <= 1e-10 and info[0].true_rel_res <= 1e-10
    xo, io = mg.mg_solve(Ho, b[0].reshape(A.V, 2), 1e-10)
    assert abs(info[0].iters - io.iters) <= 2, (info[0].iters, io.iters)
    xd = spla.spsolve(A.to_sparse().tocsc(), b[0].ravel())
    assert rel_err(psi.ravel(), xd) < 1e-6
    # CGNR comparator on the same system
    psi_c, ic = g.cgnr(dev(b), tol=1e-10)
    res_c = mg.norm(b[0].reshape(A.V, 2) - A.apply(host(psi_c)[0].reshape(A.V, 2))) / mg.norm(b)
    assert ic.converged and res_c <= 1e-10
    assert ic.iters > 5 * info[0].iters


def test_mixed_precision_solve():
    import paper_0707_4018_amd as amg
    L = 32
    U = u1_config(L, L, beta=6.0, sweeps=100, seed=4)
    m = _mcrit(U) + 0.003
    A = mg.wilson_stencil(U, m)
    init = [vectors(8, A.V, 2, 44)]
    g = amg.Gauge(dev(U), m)
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(0))
    xd = spla.spsolve(A.to_sparse().tocsc(), b[0].ravel())
    for bf16 in (False, True):
        _, pg = _params([(4, 4)], [8], inner_prec=amg.F32, p_bf16=bf16, coarse_tol=0.05, coarse_maxiter=200)
        S = amg.Solver(g, pg, init=[dev(v) for v in init])
        psi, info = S.solve(dev(b), tol=1e-10)
        psi = host(psi)[0].reshape(A.V, 2)
        res = mg.norm(b[0].reshape(A.V, 2) - A.apply(psi)) / mg.norm(b)
        assert info[0].converged and res <= 1e-10
        assert rel_err(psi.ravel(), xd) < 1e-6


def test_set_mass_equals_rebuild():
    import paper_0707_4018_amd as amg
    U, A, H, g, S = _given(16, 16, [(4, 4), (2, 2)], [4, 2], m=0.02)
    S.set_mass(0.15)
    g2 = amg.Gauge(dev(U), 0.15)
    S2 = amg.Solver(g2, S.params, nullvecs=S._keep)
    for lvl in (1, 2):
        assert max_rel_err(host(S.coarse_op(lvl)), host(S2.coarse_op(lvl))) < 1e-12


def test_multi_rhs_solve():
    U, A, H, g, S = _given(16, 16, [(4, 4)], [4], m=0.05, coarse_tol=1e-3, coarse_maxiter=100)
    b = synth.gaussian_field((3, A.V, 2, 1), synth.rng_for(10))
    psi, infos = S.solve(dev(b), tol=1e-10)
    psi = host(psi)
    for k in range(3):
        res = mg.norm(b[k].reshape(A.V, 2) - A.apply(psi[k].reshape(A.V, 2))) / mg.norm(b[k])
        assert infos[k].converged and res <= 1e-10
        p1, _ = S.solve(dev(b[k:k + 1]), tol=1e-10)
        assert rel_err(host(p1)[0], psi[k]) < 1e-8


def test_rank_error_on_duplicate_vectors():
    import paper_0707_4018_amd as amg
    U = u1_config(8, 8)
    g = amg.Gauge(dev(U), 0.1)
    v = vectors(1, 64, 2, 1)
    _, pg = _params([(4, 4)], [2])
    with pytest.raises(amg.AMGError) as e:
        amg.Solver(g, pg, nullvecs=[dev(np.concatenate([v, v]))])
    assert e.value.status == 6


def test_four_dimensional_hierarchy():
    import paper_0707_4018_amd as amg
    dims = (4, 4, 4, 4)
    U = su3_config(dims, seed=2)
    m = 0.3
    A = mg.wilson_stencil(U, m)
    po, pg = _params([(2, 2, 2, 2)], [3], coarse_tol=1e-2, coarse_maxiter=100)
    vecs = [vectors(3, A.V, 12, 5)]
    H = mg.build_hierarchy(A, vecs, po)
    g = amg.Gauge(dev(U), m)
    S = amg.Solver(g, pg, nullvecs=[dev(v) for v in vecs])
    Y = host(S.coarse_op(1))
    assert max_rel_err(Y[:, 0], H.ops[1].diag) < 1e-12
    for d in range(8):
        assert max_rel_err(Y[:, 1 + d], H.ops[1].hop[d]) < 1e-12
    b = synth.gaussian_field((1, A.V, 4, 3), synth.rng_for(11))
    psi, info = S.solve(dev(b), tol=1e-10)
    res = mg.norm(b[0].reshape(A.V, 12) - A.apply(host(psi)[0].reshape(A.V, 12))) / mg.norm(b)
    assert info[0].converged and res <= 1e-10


@pytest.mark.parametrize("case", ["2d", "4d"])
@pytest.mark.parametrize("nrhs", [1, 5, 12, 19])
def test_multi_rhs_coarse_apply_matches_oracle(case, nrhs):
    """FP32 coarse applies with several right-hand sides (MFMA kernel, rhs groups of 16
    with a ragged last group) against the FP64 Galerkin operator, rhs by rhs."""
    import torch
    import paper_0707_4018_amd as amg
    print(f"multi-rhs coarse {case} nrhs={nrhs}", flush=True)
    if case == "2d":
        U, A, H, g, S = _given(16, 32, [(4, 4)], [8])
        pg = S.params
    else:
        dims = (8, 4, 4, 8)
        U = su3_config(dims, seed=6, smear=2)
        A = mg.wilson_stencil(U, 0.2)
        vecs = [vectors(24, A.V, 12, 17)]
        po, pg = _params([(4, 4, 4, 4)], [24])
        H = mg.build_hierarchy(A, vecs, po)
        g = amg.Gauge(dev(U), 0.2)
        S = amg.Solver(g, pg, nullvecs=[dev(v) for v in vecs])
    pg.inner_prec = amg.F32
    S32 = amg.Solver(g, pg, nullvecs=S._keep)
    Ac = H.ops[1]
    e = synth.gaussian_field((nrhs, Ac.V, Ac.dof), synth.rng_for(12, nrhs))
    for dag in (False, True):
        out = host(S32.level_apply(1, dev(e, torch.complex64), dagger=dag, prec=amg.F32, nrhs=nrhs))
        for r in range(nrhs):
            ref = Ac.apply_dagger(e[r]) if dag else Ac.apply(e[r])
            assert rel_err(out[r], ref) < 2e-5, (dag, r)


@pytest.mark.parametrize("nrhs", [1, 3, 5, 12, 17])
def test_four_dimensional_transfers_match_oracle(nrhs):
    """Restriction / prolongation with 4^4 blocks and 24 vectors (the per-wave kernels with
    right-hand sides grouped inside the wave) against the oracle, rhs by rhs; the coarse
    operator built from them matches the sparse triple product."""
    import paper_0707_4018_amd as amg
    print(f"4d transfers nrhs={nrhs}", flush=True)
    dims = (8, 4, 4, 8)
    U = su3_config(dims, seed=8, smear=2)
    A = mg.wilson_stencil(U, 0.3)
    vecs = [vectors(24, A.V, 12, 19)]
    po, pg = _params([(4, 4, 4, 4)], [24])
    H = mg.build_hierarchy(A, vecs, po)
    S = amg.Solver(amg.Gauge(dev(U), 0.3), pg, nullvecs=[dev(v) for v in vecs])
    P = H.Ps[0]
    r = synth.gaussian_field((nrhs, A.V, 4, 3), synth.rng_for(13, nrhs))
    rc = host(S.restrict(0, dev(r), nrhs=nrhs))
    e = synth.gaussian_field((nrhs, P.Vc, P.nc), synth.rng_for(14, nrhs))
    pe = host(S.prolong(0, dev(e), nrhs=nrhs))
    for i in range(nrhs):
        assert max_rel_err(rc[i], P.restrict(r[i].reshape(A.V, 12))) < 1e-12
        assert max_rel_err(pe[i].reshape(A.V, 12), P.prolong(e[i])) < 1e-12


@pytest.mark.parametrize("L1,L2", [(128, 128), (132, 128), (160, 160), (512, 512)])
def test_mr_reductions_across_grid_sizes(L1, L2):
    """MR on the fine level needs <p, r> and <p, p> over the whole lattice in
    every step: 64 blocks (one ticket level), 66 and 100 blocks (two levels,
    ragged last group) and the 1024-block cap; bitwise reproducible."""
    import paper_0707_4018_amd as amg
    print(f"fine MR reductions {L1}x{L2}", flush=True)
    U = u1_config(L1, L2, sweeps=10)
    A = mg.wilson_stencil(U, 0.05)
    g = amg.Gauge(dev(U), 0.05)
    S = amg.Solver(g, amg.MGParams(blocks=[(4, 4)], nvec=[4]), nullvecs=[dev(vectors(4, A.V, 2, 11))])
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(12, L1, L2))
    x1 = host(S.mr(0, 3, dev(b)))
    x2 = host(S.mr(0, 3, dev(b)))
    assert np.array_equal(x1, x2)
    xo = mg.mr(A, b[0].reshape(A.V, 2), 3, 0.8)[0]
    assert max_rel_err(x1.reshape(-1), xo.reshape(-1)) < 1e-12


@pytest.mark.parametrize("nrhs", [1, 3, 5, 12])
def test_four_dimensional_fp32_mr_multi_rhs(nrhs):
    """FP32 MR on the 4d fine level (stencil with the MR sums in its epilogue,
    one launch over all right-hand sides) against the FP64 oracle MR, and
    against the same MR run one rhs at a time."""
    import torch
    import paper_0707_4018_amd as amg
    print(f"4d fp32 MR nrhs={nrhs}", flush=True)
    dims = (8, 4, 4, 8)
    U = su3_config(dims, seed=9, smear=2)
    m = 0.1
    A = mg.wilson_stencil(U, m)
    _, pg = _params([(4, 4, 4, 4)], [6], inner_prec=amg.F32)
    S = amg.Solver(amg.Gauge(dev(U), m), pg, nullvecs=[dev(vectors(6, A.V, 12, 23))])
    b = synth.gaussian_field((nrhs, A.V, 4, 3), synth.rng_for(15, nrhs))
    x = host(S.mr(0, 3, dev(b, torch.complex64), nrhs=nrhs, prec=amg.F32))
    for r in range(nrhs):
        xo = mg.mr(A, b[r].reshape(A.V, 12), 3, 0.8)[0]
        assert rel_err(x[r].reshape(-1), xo.reshape(-1)) < 1e-5, r
        x1 = host(S.mr(0, 3, dev(b[r:r + 1], torch.complex64), prec=amg.F32))
        assert rel_err(x[r].reshape(-1), x1.reshape(-1)) < 1e-6, r


def test_large_lattice_mixed_solve():
    """A 1024^2 mixed-precision adaptive solve.  At this size the fine-level
    residual of the V-cycle (FP32), the outer FGCR residual (FP64) and the
    setup's error propagation (FP64) run the x_2-marching stencil with the
    residual epilogue; the true residual is recomputed with the oracle's D."""
    import paper_0707_4018_amd as amg
    L = 1024
    print(f"mixed solve {L}x{L}", flush=True)
    th = synth.u1_heatbath(8, 8, 6.0, 20, synth.rng_for(90, 600, 8, 8, 11))
    U = np.exp(1j * synth.tile_u1(th, L // 8, L // 8))[..., None, None]
    m = 0.1
    A = mg.wilson_stencil(U, m)
    g = amg.Gauge(dev(U), m)
    _, pg = _params([(4, 4)], [8], inner_prec=amg.F32, p_bf16=True, coarse_tol=0.1, coarse_maxiter=100)
    S = amg.Solver(g, pg, init=[dev(vectors(8, A.V, 2, 46))])
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(16, L))
    psi, info = S.solve(dev(b), tol=1e-10)
    res = mg.norm(b[0].reshape(A.V, 2) - A.apply(host(psi)[0].reshape(A.V, 2))) / mg.norm(b)
    assert info[0].converged and res <= 1e-10


def test_non_finite_rhs_is_rejected():
    """A right-hand side with a NaN or an infinite entry: AMG_ERR_NAN before any
    iteration; the solver then solves a clean system as before."""
    import paper_0707_4018_amd as amg
    print("non-finite rhs", flush=True)
    U, A, H, g, S = _given(16, 16, [(4, 4)], [4])
    b = synth.gaussian_field((3, A.V, 2, 1), synth.rng_for(18))
    x_ref, _ = S.solve(dev(b), tol=1e-10)
    for bad in (np.nan, np.inf):
        bb = b.copy()
        bb[1, 7, 0, 0] = bad
        with pytest.raises(amg.AMGError) as e:
            S.solve(dev(bb), tol=1e-10)
        assert e.value.status == 3
    x, info = S.solve(dev(b), tol=1e-10)
    assert all(i.converged for i in info)
    assert np.array_equal(host(x), host(x_ref))


@pytest.mark.parametrize("L1,L2", [(1024, 1024), (1024, 1032)])
def test_mr_on_streaming_size_lattices(L1, L2):
    """MR on a fine lattice of 2^20 sites and more: the stencil with the MR sums
    marches along x_2 (1024^2, tile-strided capped grid) or runs one site per
    thread (1024 x 1032); FP64 and FP32 against the oracle's MR, bitwise
    reproducible."""
    import torch
    import paper_0707_4018_amd as amg
    print(f"fine MR {L1}x{L2}", flush=True)
    th = synth.u1_heatbath(8, 8, 6.0, 20, synth.rng_for(90, 600, 8, 8, 13))
    U = np.exp(1j * synth.tile_u1(th, L1 // 8, L2 // 8))[..., None, None]
    m = 0.05
    A = mg.wilson_stencil(U, m)
    g = amg.Gauge(dev(U), m)
    _, pg = _params([(4, 4)], [4], inner_prec=amg.F32)
    S = amg.Solver(g, pg, nullvecs=[dev(vectors(4, A.V, 2, 47))])
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(19, L1, L2))
    xo = mg.mr(A, b[0].reshape(A.V, 2), 3, 0.8)[0]
    x1 = host(S.mr(0, 3, dev(b)))
    assert np.array_equal(x1, host(S.mr(0, 3, dev(b))))
    assert max_rel_err(x1.reshape(-1), xo.reshape(-1)) < 1e-12
    x32 = host(S.mr(0, 3, dev(b, torch.complex64), prec=amg.F32))
    assert rel_err(x32.reshape(-1), xo.reshape(-1)) < 1e-5


def _bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned widened."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def _rounded_prolongator(P: "mg.Prolongator", Q: np.ndarray) -> "mg.Prolongator":
    return mg.Prolongator(P.fine_dims, P.block, P.dof, P.nvec, Q, P.blk)


@pytest.mark.parametrize("case,bf16", [("2d", False), ("2d", True), ("4d", False), ("4d", True)])
def test_fp32_transfers_match_oracle_on_stored_prolongator(case, bf16):
    """FP32 restriction / prolongation (the kernels of the FP32 cycle, P in FP32
    or bfloat16) element by element against the oracle's transfers built on
    the prolongator the library stores; the stored P itself is the oracle's
    FP64 P rounded (bit-exactly for the bfloat16 rounding of the library's
    FP64 P)."""
    import torch
    import paper_0707_4018_amd as amg
    print(f"fp32 transfers {case} bf16={bf16}", flush=True)
    if case == "2d":
        dims, block, nv, dof = (32, 16), (4, 4), 8, 2
        U = u1_config(*dims)
        rhs_list = [1, 3]
    else:
        dims, block, nv, dof = (8, 4, 4, 8), (4, 4, 4, 4), 24, 12
        U = su3_config(dims, seed=10, smear=2)
        rhs_list = [1, 5, 12]
    A = mg.wilson_stencil(U, 0.1)
    vecs = [vectors(nv, A.V, dof, 61)]
    po, pg = _params([block], [nv], inner_prec=amg.F32, p_bf16=bf16)
    H = mg.build_hierarchy(A, vecs, po)
    S = amg.Solver(amg.Gauge(dev(U), 0.1), pg, nullvecs=[dev(v) for v in vecs])
    P64 = host(S.prolongator(0, amg.F64))
    P32 = host(S.prolongator(0, amg.F32))
    if bf16:
        # with bfloat16 storage the library rounds its FP64 P as well (the
        # Galerkin operator is built from the P the transfers use): the FP64
        # copy lies on the bfloat16 grid, within one bfloat16 step of the
        # oracle's P, and the stored copy holds the same values
        on_grid = _bf16_round(P64.real.astype(np.float32)) + 1j * _bf16_round(P64.imag.astype(np.float32))
        assert np.array_equal(P64, on_grid.astype(np.complex128))
        assert np.abs(P64 - H.Ps[0].Q).max() <= 2.0 ** -8 * np.abs(H.Ps[0].Q).max()
        assert np.array_equal(P32, P64)
    else:
        assert max_rel_err(P64, H.Ps[0].Q) < 1e-12
        ref = P64.real.astype(np.float32) + 1j * P64.imag.astype(np.float32)
        assert np.array_equal(P32, ref.astype(np.complex128))
    Pr = _rounded_prolongator(H.Ps[0], P32)
    ns, nc = (2, 1) if case == "2d" else (4, 3)
    for nrhs in rhs_list:
        r = synth.gaussian_field((nrhs, A.V, ns, nc), synth.rng_for(62, nrhs))
        e = synth.gaussian_field((nrhs, Pr.Vc, Pr.nc), synth.rng_for(63, nrhs))
        r32 = r.astype(np.complex64)
        e32 = e.astype(np.complex64)
        rc = host(S.restrict(0, dev(r32), nrhs=nrhs, prec=amg.F32))
        pe = host(S.prolong(0, dev(e32), nrhs=nrhs, prec=amg.F32))
        for i in range(nrhs):
            ro = Pr.restrict(r32[i].astype(np.complex128).reshape(A.V, dof))
            po_ = Pr.prolong(e32[i].astype(np.complex128))
            assert max_rel_err(rc[i], ro) < 2e-6, (nrhs, i)
            assert max_rel_err(pe[i].reshape(A.V, dof), po_) < 2e-6, (nrhs, i)


class _Wilson4dOp:
    """The oracle's D (the formula, dirac.apply_D) for fields of shape (V, 12):
    what mg.mr needs, without the per-site block matrices of a Stencil."""

    def __init__(self, U, m):
        from oracle import dirac
        self.U, self.m, self.dirac = U, m, dirac
        self.lat = U.shape[1:5]
        self.V = int(np.prod(self.lat))

    def apply(self, f):
        return self.dirac.apply_D(self.U, f.reshape(self.lat + (4, 3)), self.m).reshape(self.V, 12)


@pytest.mark.parametrize("nrhs", [1, 12])
def test_four_dimensional_fp32_mr_multi_slab(nrhs):
    """FP32 MR on a 16^3 x 64 fine level: the stencil with the MR sums marches
    x_4 in four slabs of 16 sites, 64 blocks per rhs renumbered by XCD, with
    the grid reduction across them; against the oracle's MR on its D."""
    import torch
    import paper_0707_4018_amd as amg
    print(f"4d fp32 MR 16^3x64 nrhs={nrhs}", flush=True)
    base, tile = (8, 8, 8, 8), (2, 2, 2, 8)
    dims = tuple(b * t for b, t in zip(base, tile))
    U = np.tile(su3_config(base, seed=12, smear=2), (1,) + tuple(reversed(tile)) + (1, 1))
    m = 0.1
    V = int(np.prod(dims))
    _, pg = _params([(4, 4, 4, 4)], [2], inner_prec=amg.F32)
    vv = synth.gaussian_field((2, V, 12), synth.rng_for(64))
    S = amg.Solver(amg.Gauge(dev(U), m), pg, nullvecs=[dev(vv)])
    b = synth.gaussian_field((nrhs, V, 4, 3), synth.rng_for(65, nrhs))
    x = host(S.mr(0, 3, dev(b, torch.complex64), nrhs=nrhs, prec=amg.F32))
    Aop = _Wilson4dOp(U, m)
    for r in ([0, nrhs - 1] if nrhs > 1 else [0]):
        xo = mg.mr(Aop, b[r].reshape(V, 12), 3, 0.8)[0]
        assert max_rel_err(x[r].reshape(-1), xo.reshape(-1)) < 1e-5, r


@pytest.mark.parametrize("dense", [4096, 0])
def test_three_level_adaptive_vectors_match_oracle(dense):
    """Adaptive setup on three levels (32^2 -> 8^2 -> 4^2): the vectors of both
    coarsenings equal the oracle's from the same random starts."""
    import paper_0707_4018_amd as amg
    print(f"3-level adaptive vectors dense={dense}", flush=True)
    U = u1_config(32, 32, beta=6.0, sweeps=60, seed=5)
    m = 0.03
    A = mg.wilson_stencil(U, m)
    po, pg = _params([(4, 4), (2, 2)], [4, 4], coarse_tol=0.05, coarse_maxiter=60, coarse_restart=16,
                     coarse_dense_max=dense)
    init = [vectors(4, A.V, 2, 71), vectors(4, 64, 8, 72)]
    Ho, vo = mg.adaptive_setup(A, po, init, nu0=10, ncyc=2)
    S = amg.Solver(amg.Gauge(dev(U), m), pg, init=[dev(v) for v in init], nu0=10, ncyc=2)
    for lvl in range(2):
        v = host(S.nullvecs(lvl))
        assert rel_err(v, vo[lvl]) < 1e-7, lvl
    Y2 = host(S.coarse_op(2))
    assert max_rel_err(Y2[:, 0], Ho.ops[2].diag) < 1e-7


def test_level_apply_fp32_on_fp64_solver_grows_buffers():
    """FP32 fine-level applies on an FP64 solver, first with one right-hand side
    and then with four (the FP32 work buffers must grow), against the oracle."""
    import torch
    import paper_0707_4018_amd as amg
    from oracle import dirac
    print("level_apply fp32 on fp64 solver, nrhs 1 then 4", flush=True)
    U, A, H, g, S = _given(16, 16, [(4, 4)], [4])
    for nrhs in (1, 4):
        psi = synth.gaussian_field((nrhs, A.V, 2, 1), synth.rng_for(66, nrhs))
        out = host(S.level_apply(0, dev(psi, torch.complex64), prec=amg.F32, nrhs=nrhs))
        for k in range(nrhs):
            ref = dirac.apply_D(U, psi[k].reshape(16, 16, 2, 1), 0.05).reshape(-1, 2, 1)
            assert max_rel_err(out[k], ref) < 1e-5, (nrhs, k)


@pytest.mark.parametrize("nv", [3, 24])
def test_four_dimensional_block_jacobi_vcycle_matches_oracle(nv):
    """4d coarsest GCR with the block-Jacobi preconditioner (no even-odd
    reduction in 4d): 6 and 48 coarse dof per site (the 48-wide block
    inverse), 10 steps with restart 5 on both sides, then a solve to 1e-10."""
    import paper_0707_4018_amd as amg
    print(f"4d block-jacobi vcycle nv={nv}", flush=True)
    dims = (4, 4, 4, 4)
    U = su3_config(dims, seed=2)
    m = 0.3
    A = mg.wilson_stencil(U, m)
    po, pg = _params([(2, 2, 2, 2)], [nv], coarse_tol=0.0, coarse_maxiter=10, coarse_restart=5, coarse_dense_max=0,
                     coarse_jacobi=True)
    vecs = [vectors(nv, A.V, 12, 5)]
    H = mg.build_hierarchy(A, vecs, po)
    S = amg.Solver(amg.Gauge(dev(U), m), pg, nullvecs=[dev(v) for v in vecs])
    b = synth.gaussian_field((1, A.V, 4, 3), synth.rng_for(12))
    x = host(S.vcycle(dev(b)))[0].reshape(A.V, 12)
    assert rel_err(x, mg.vcycle(H, 0, b[0].reshape(A.V, 12))) < 1e-10
    pg.coarse_tol = 0.1
    S2 = amg.Solver(amg.Gauge(dev(U), m), pg, nullvecs=[dev(v) for v in vecs])
    psi, info = S2.solve(dev(b), tol=1e-10)
    res = mg.norm(b[0].reshape(A.V, 12) - A.apply(host(psi)[0].reshape(A.V, 12))) / mg.norm(b)
    assert info[0].converged and res <= 1e-10


def test_even_odd_option_edges():
    """coarse_eo without coarse_jacobi is rejected; a coarse lattice with odd
    extents (20^2 / 4^2 = 5^2) keeps the block-Jacobi GCR without the
    reduction, like the oracle, and the cycle still matches it."""
    import paper_0707_4018_amd as amg
    print("even-odd option edges", flush=True)
    U = u1_config(20, 20, seed=4)
    _, pg = _params([(4, 4)], [4], coarse_eo=True)
    with pytest.raises(amg.AMGError) as e:
        amg.Solver(amg.Gauge(dev(U), 0.05), pg, nullvecs=[dev(vectors(4, 400, 2, 3))])
    assert e.value.status == 1
    U, A, H, g, S = _given(20, 20, [(4, 4)], [4], m=0.05, coarse_tol=0.0, coarse_maxiter=8, coarse_restart=4,
                           coarse_dense_max=0, coarse_jacobi=True, coarse_eo=True)
    b = synth.gaussian_field((1, A.V, 2, 1), synth.rng_for(14))
    x = host(S.vcycle(dev(b)))[0].reshape(A.V, 2)
    assert rel_err(x, mg.vcycle(H, 0, b[0].reshape(A.V, 2))) < 1e-10
