"""Pins of the oracle's multigrid pieces.

Every check compares the oracle with something it does not compute the same
way: a sparse-matrix product for the Galerkin operator (Eq. (2)), dense
linear algebra for exact solves and exact coarse corrections, the operator
form of the V-cycle (Eq. (3), with the sign of the R A R^dagger term read as
minus), algebraic identities of the chirally split prolongator, and
monotonicity properties of MR and GCR.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import dirac, mg


def _field(L1, L2, beta=6.0, sweeps=30, seed=0):
    th = synth.u1_heatbath(L1, L2, beta, sweeps, synth.rng_for(96, seed, L1, L2))
    return dirac.u1_field(th)


def _vecs(n, V, dof, seed):
    return np.stack([synth.gaussian_field((V, dof), synth.rng_for(95, seed, k)) for k in range(n)])


def _setup(L1, L2, block, nv, m=0.1, seed=0):
    U = _field(L1, L2, seed=seed)
    A = mg.wilson_stencil(U, m)
    v = np.stack([mg.relax_homogeneous(A, x, 10, 0.8) for x in _vecs(nv, A.V, 2, seed)])
    P = mg.build_prolongator(v, A.dims, block)
    return A, P, v


@pytest.mark.parametrize("L1,L2,block,nv", [(8, 8, (4, 4), 4), (4, 4, (4, 4), 3),
                                           (16, 8, (4, 4), 4), (12, 8, (4, 2), 2)])
def test_prolongator_identities(L1, L2, block, nv):
    A, P, v = _setup(L1, L2, block, nv)
    Ps = P.to_sparse().toarray()
    assert np.abs(Ps.conj().T @ Ps - np.eye(Ps.shape[1])).max() < 1e-13        # P^dag P = 1
    for k in range(nv):                                                          # P P^dag v_k = v_k
        vk = v[k]
        assert mg.norm(P.prolong(P.restrict(vk)) - vk) < 1e-12 * mg.norm(vk)
    g5f = np.tile(mg.gamma5_diag(2), A.V)
    g5c = np.tile(mg.gamma5_diag(P.nc), P.Vc)
    assert np.abs(g5f[:, None] * Ps - Ps * g5c[None, :]).max() < 1e-14           # gamma5 P = P Gamma5
    # restriction is the adjoint of prolongation
    e = synth.gaussian_field((P.Vc, P.nc), synth.rng_for(1))
    r = synth.gaussian_field((A.V, 2), synth.rng_for(2))
    assert abs(mg.vdot(P.prolong(e), r) - mg.vdot(e, P.restrict(r))) < 1e-12


@pytest.mark.parametrize("L1,L2,block,nv", [(8, 8, (4, 4), 4), (4, 4, (4, 4), 3),
                                           (16, 8, (4, 4), 2), (12, 8, (4, 2), 3),
                                           (8, 8, (2, 2), 2)])
def test_galerkin_equals_sparse_triple_product(L1, L2, block, nv):
    A, P, _ = _setup(L1, L2, block, nv)
    Ac = mg.galerkin(A, P)
    Ps = P.to_sparse()
    ref = (Ps.conj().T @ A.to_sparse() @ Ps).toarray()
    assert np.abs(Ac.to_sparse().toarray() - ref).max() < 1e-13
    # coarse gamma5-hermiticity: Gamma5 D_hat Gamma5 = D_hat^dagger
    g5c = np.tile(mg.gamma5_diag(P.nc), P.Vc)
    M = Ac.to_sparse().toarray()
    assert np.abs(g5c[:, None] * M * g5c[None, :] - M.conj().T).max() < 1e-13
    # coarse dagger apply agrees with the matrix adjoint
    e = synth.gaussian_field((P.Vc, P.nc), synth.rng_for(3))
    assert np.abs(Ac.apply_dagger(e).ravel() - M.conj().T @ e.ravel()).max() < 1e-12


def test_galerkin_4d():
    dims = (4, 4, 2, 4)
    U = synth.su3_haar((4,) + tuple(reversed(dims)), synth.rng_for(77))
    A = mg.wilson_stencil(U, 0.3)
    v = _vecs(2, A.V, 12, 5)
    P = mg.build_prolongator(v, dims, (2, 2, 2, 2))
    Ps = P.to_sparse()
    ref = (Ps.conj().T @ A.to_sparse() @ Ps).toarray()
    assert np.abs(mg.galerkin(A, P).to_sparse().toarray() - ref).max() < 1e-12


def test_three_level_and_mass_reuse():
    U = _field(16, 16)
    A = mg.wilson_stencil(U, 0.05)
    p = mg.MGParams(blocks=[(4, 4), (2, 2)], nvec=[3, 2])
    v0 = _vecs(3, A.V, 2, 9)
    A1_tmp = mg.galerkin(A, mg.build_prolongator(v0, A.dims, (4, 4)))
    v1 = _vecs(2, A1_tmp.V, A1_tmp.dof, 10)
    H = mg.build_hierarchy(A, [v0, v1], p)
    P1, P2 = H.Ps[0].to_sparse(), H.Ps[1].to_sparse()
    ref = (P2.conj().T @ P1.conj().T @ A.to_sparse() @ P1 @ P2).toarray()
    assert np.abs(H.ops[2].to_sparse().toarray() - ref).max() < 1e-12
    # reusing the setup at a heavier mass equals rebuilding at that mass
    H2 = mg.with_mass(H, 0.2)
    Hb = mg.build_hierarchy(mg.wilson_stencil(U, 0.25), [v0, v1], p)
    for a, b in zip(H2.ops, Hb.ops):
        assert np.abs(a.to_sparse() - b.to_sparse()).max() < 1e-12


def test_exact_two_grid_correction_is_galerkin_orthogonal():
    A, P, _ = _setup(8, 8, (4, 4), 4)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(4))
    x, _ = mg.mr(A, b, 2, 0.8)
    Ac = mg.galerkin(A, P)
    Mc = Ac.to_sparse().toarray()
    ec = np.linalg.solve(Mc, P.restrict(b - A.apply(x)).ravel()).reshape(P.Vc, P.nc)
    x2 = x + P.prolong(ec)
    assert mg.norm(P.restrict(b - A.apply(x2))) < 1e-12 * mg.norm(b)


def test_vcycle_operator_formula_sign():
    """With a linear (Richardson) smoother R = R^dag = w 1 and an exact coarse solve,
    the five-step V-cycle equals R + R^dag - R A R^dag + (1 - R A) P Vc P^dag (1 - A R^dag),
    and not the printed '+ R A R^dag' variant."""
    A, P, _ = _setup(4, 4, (2, 2), 2)
    w = 0.3

    def richardson(Aop, b, nu, omega):
        x = w * b
        return x, b - Aop.apply(x)

    Ac = mg.galerkin(A, P)
    p = mg.MGParams(blocks=[(2, 2)], nvec=[2], nu_pre=1, nu_post=1, coarse_tol=1e-15,
                    coarse_maxiter=500, coarse_restart=500, smoother=richardson)
    H = mg.Hierarchy([A, Ac], [P], p)
    N = A.V * A.dof
    Vmat = np.zeros((N, N), dtype=np.complex128)
    for i in range(N):
        e = np.zeros(N, dtype=np.complex128)
        e[i] = 1.0
        Vmat[:, i] = mg.vcycle(H, 0, e.reshape(A.V, A.dof)).ravel()
    Am = A.to_sparse().toarray()
    Pm = P.to_sparse().toarray()
    Vc = np.linalg.inv(Pm.conj().T @ Am @ Pm)
    R = w * np.eye(N)
    I = np.eye(N)
    corr = (I - R @ Am) @ Pm @ Vc @ Pm.conj().T @ (I - Am @ R)
    minus = R + R - R @ Am @ R + corr
    plus = R + R + R @ Am @ R + corr
    assert np.abs(Vmat - minus).max() < 1e-10
    assert np.abs(Vmat - plus).max() > 1e-2


def test_mr_residual_monotone_and_consistent():
    A, _, _ = _setup(8, 8, (4, 4), 1)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(5))
    last = mg.norm(b)
    for nu in range(1, 6):
        x, r = mg.mr(A, b, nu, 0.8)
        assert mg.norm(r - (b - A.apply(x))) < 1e-12 * mg.norm(b)
        assert mg.norm(r) <= last + 1e-14
        last = mg.norm(r)


def test_fgcr_matches_dense_solve_and_is_monotone():
    U = _field(8, 8)
    A = mg.wilson_stencil(U, 0.1)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(6))
    x, info = mg.fgcr(A, b, lambda r: r, 1e-12, 2000, 8)
    assert info.converged
    xd = np.linalg.solve(dirac.dense_D(U, 0.1), b.ravel())
    kappa = np.linalg.cond(dirac.dense_D(U, 0.1))
    assert mg.norm(x.ravel() - xd) <= kappa * 1e-12 * mg.norm(xd) * 10
    h = info.history
    # within each restart cycle of 8, the recursive residual never grows
    for start in range(0, len(h) - 1, 9):
        seg = h[start:start + 9]
        assert all(seg[i + 1] <= seg[i] * (1 + 1e-12) for i in range(len(seg) - 1))


@pytest.mark.parametrize("L", [8, 16])
def test_mg_solve_matches_direct_solve(L):
    U = _field(L, L, seed=1)
    m = 0.05
    A = mg.wilson_stencil(U, m)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(7, L))
    p = mg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_tol=1e-12, coarse_maxiter=1000, coarse_restart=64)
    init = [_vecs(4, A.V, 2, 8)]
    H, _ = mg.adaptive_setup(A, p, init)
    x, info = mg.mg_solve(H, b, 1e-10)
    assert info.converged and info.true_rel_res <= 1e-10
    xd = spla.spsolve(A.to_sparse().tocsc(), b.ravel())
    assert mg.norm(x.ravel() - xd) < 1e-7 * mg.norm(xd)


def test_cgnr_converges_on_original_residual():
    U = _field(8, 8)
    A = mg.wilson_stencil(U, 0.1)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(9))
    n0 = A.napply
    x, info = mg.cgnr(A, b, 1e-10, 5000)
    assert info.converged
    assert A.napply - n0 == 2 * info.iters + 2       # one D and one D^dag per iteration (+ setup, check)


def test_rank_error_on_duplicate_vectors():
    U = _field(8, 8)
    A = mg.wilson_stencil(U, 0.1)
    v = _vecs(1, A.V, 2, 3)
    with pytest.raises(mg.RankError):
        mg.build_prolongator(np.concatenate([v, v]), A.dims, (4, 4))


def test_adaptive_setup_finds_near_null_space():
    """Adaptive vectors have a much smaller Rayleigh quotient than random ones,
    and the MG iteration count barely moves as the mass approaches critical."""
    L = 16
    U = _field(L, L, seed=2)
    e0 = np.linalg.eigvals(dirac.dense_D(U, 0.0))
    mcrit = -e0.real.min()
    p = mg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_tol=1e-12, coarse_maxiter=1000, coarse_restart=64)
    A = mg.wilson_stencil(U, mcrit + 0.01)
    init = [_vecs(4, A.V, 2, 11)]
    H, vecs = mg.adaptive_setup(A, p, init)
    rq = [mg.norm(A.apply(v)) / mg.norm(v) for v in vecs[0]]
    rq0 = [mg.norm(A.apply(v)) / mg.norm(v) for v in init[0]]
    assert max(rq) < 0.5 * min(rq0)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(12))
    its = []
    for dm in (0.09, 0.0):
        x, info = mg.mg_solve(mg.with_mass(H, dm), b, 1e-10)
        assert info.converged
        its.append(info.iters)
    assert its[1] <= its[0] + 6
