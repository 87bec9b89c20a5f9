"""Pins of the oracle's multigrid for the normal equations A = D^dagger D.

Against what the paper and linear algebra fix: the V-cycle with R = R^dagger
and an exact coarsest solve is Hermitian and positive definite (Eq. (3)) and
equals the operator formula term by term; the frozen smoother is the
polynomial its two step lengths define; a minimal-residual step minimises
the residual; the prolongator is orthonormal and reproduces its vectors;
(MG-)CG reaches the sparse direct solution.
"""
import numpy as np
import scipy.sparse.linalg as spla

import synth
from oracle import dirac, mg, normal


def _field(L, beta=6.0, sweeps=40, seed=0):
    th = synth.u1_heatbath(L, L, beta, sweeps, synth.rng_for(120, seed, L))
    return dirac.u1_field(th)


def _D(L, m, seed=0):
    return mg.wilson_stencil(_field(L, seed=seed), m).to_sparse()


def _vecs(n, V, dof, seed):
    return np.stack([synth.gaussian_field((V, dof), synth.rng_for(121, seed, k)) for k in range(n)])


def _hier(L, blocks, nvec, m=0.05, seed=0):
    D = _D(L, m, seed)
    dims = [(L, L)]
    vecs, sb = [], []
    for l, (b, nv) in enumerate(zip(blocks, nvec)):
        V = dims[-1][0] * dims[-1][1]
        dof = 2 if l == 0 else nvec[l - 1]
        vecs.append(_vecs(nv, V, dof, seed * 10 + l))
        sb.append(synth.gaussian_field((V * dof,), synth.rng_for(122, seed, l)))
        dims.append((dims[-1][0] // b[0], dims[-1][1] // b[1]))
    V = dims[0][0] * dims[0][1]
    return D, normal.build(D, (L, L), vecs, blocks, sb), vecs


def test_prolongator_orthonormal_and_keeps_vectors():
    D, H, vecs = _hier(16, [(4, 4)], [4])
    P = H.Ps[0]
    assert abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-13
    for v in vecs[0]:
        vv = v.reshape(-1)
        assert np.linalg.norm(P @ (P.conj().T @ vv) - vv) < 1e-12 * np.linalg.norm(vv)


def test_coarse_operators_hermitian_positive_definite():
    D, H, _ = _hier(16, [(4, 4), (2, 2)], [4, 3])
    for A in H.ops:
        M = A.M.toarray()
        assert np.abs(M - M.conj().T).max() < 1e-12 * np.abs(M).max()
        assert np.linalg.eigvalsh(M).min() > 0


def test_frozen_step_minimises_the_residual():
    """With omega = 1 the first step length is the minimal-residual one:
    |b - t A b| is smallest at t = tau_0."""
    D, H, _ = _hier(8, [(4, 4)], [2])
    A = H.ops[0]
    b = synth.gaussian_field((A.n,), synth.rng_for(123))
    t0, _ = normal.frozen_steps(A, b, 1.0)
    f = lambda t: np.linalg.norm(b - t * A.apply(b))  # noqa: E731
    for d in (1e-3, -1e-3, 1e-2, -1e-2):
        assert f(t0) < f(t0 + d * abs(t0))


def test_smoother_is_its_polynomial():
    """x = R b with R = (tau0 + tau1) - tau0 tau1 A, and the tracked residual
    is (1 - tau1 A)(1 - tau0 A) b."""
    D, H, _ = _hier(8, [(4, 4)], [2])
    A = H.ops[0]
    M = A.M.toarray()
    t0, t1 = H.taus[0]
    b = synth.gaussian_field((A.n,), synth.rng_for(124))
    x, r = normal.smooth(A, b, (t0, t1))
    R = (t0 + t1) * np.eye(A.n) - t0 * t1 * M
    assert np.linalg.norm(x - R @ b) < 1e-12 * np.linalg.norm(x)
    I = np.eye(A.n)
    assert np.linalg.norm(r - (I - t1 * M) @ (I - t0 * M) @ b) < 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(normal.smooth_add(A, b, (t0, t1)) - R @ b) < 1e-12 * np.linalg.norm(x)


def _vcycle_matrix(H):
    n = H.ops[0].n
    V = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[i] = 1.0
        V[:, i] = normal.vcycle(H, 0, e)
    return V


def test_vcycle_equals_operator_formula():
    """Eq. (3) with R = R^dagger and the coarse term's sign read as minus:
    V = R + R^dag - R A R^dag + (1 - R A) P A_c^-1 P^dag (1 - A R^dag)."""
    D, H, _ = _hier(8, [(4, 4)], [3])
    V = _vcycle_matrix(H)
    A = H.ops[0].M.toarray()
    P = H.Ps[0].toarray()
    Ac = H.ops[1].M.toarray()
    t0, t1 = H.taus[0]
    n = A.shape[0]
    I = np.eye(n)
    R = (t0 + t1) * I - t0 * t1 * A
    ref = R + R.conj().T - R @ A @ R.conj().T + (I - R @ A) @ P @ np.linalg.inv(Ac) @ P.conj().T @ (I - A @ R.conj().T)
    assert np.abs(V - ref).max() < 1e-10 * np.abs(ref).max()


def test_three_level_vcycle_hermitian_positive_definite():
    """<x, V y> = <V x, y> and <x, V x> > 0 on three levels (Eq. (3))."""
    D, H, _ = _hier(32, [(4, 4), (4, 4)], [4, 4])
    n = H.ops[0].n
    for s in range(3):
        x = synth.gaussian_field((n,), synth.rng_for(125, s))
        y = synth.gaussian_field((n,), synth.rng_for(126, s))
        Vx, Vy = normal.vcycle(H, 0, x), normal.vcycle(H, 0, y)
        lhs, rhs = normal.vdot(x, Vy), normal.vdot(Vx, y)
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)
        assert normal.vdot(x, Vx).real > 0 and abs(normal.vdot(x, Vx).imag) < 1e-11 * abs(normal.vdot(x, Vx))


def test_pcg_and_mgcg_reach_the_direct_solution():
    D, H, _ = _hier(16, [(4, 4)], [4])
    A = H.ops[0]
    chi = synth.gaussian_field((A.n,), synth.rng_for(127))
    b = D.conj().T @ chi
    xd = spla.spsolve(A.M.tocsc(), b)
    x, info = normal.pcg(A, b, None, 1e-12, 5000)
    assert info.converged and np.linalg.norm(x - xd) < 1e-8 * np.linalg.norm(xd)
    x2, info2 = normal.mgcg(H, b, 1e-12)
    assert info2.converged and np.linalg.norm(x2 - xd) < 1e-8 * np.linalg.norm(xd)
    assert info2.iters < info.iters
    # the solution of the normal equations solves D psi = chi
    assert np.linalg.norm(chi - D @ x2) < 1e-9 * np.linalg.norm(chi) * 1e3
    # an exact preconditioner: one iteration
    lu = spla.splu(A.M.tocsc())
    _, info3 = normal.pcg(A, b, lu.solve, 1e-12, 10)
    assert info3.iters == 1


def test_adaptive_vectors_beat_random_ones():
    """The adaptive vectors (Eq. (4) and the V-cycle passes after it) have
    smaller Rayleigh quotients |A v|/|v| than the random vectors they start
    from, and MG-CG with them needs fewer iterations than with a prolongator
    built from the random vectors themselves."""
    L = 16
    th = synth.u1_heatbath(L, L, 6.0, 60, synth.rng_for(128, L))
    U = dirac.u1_field(th)
    mcrit = -np.linalg.eigvals(dirac.dense_D(U, 0.0)).real.min()
    D = mg.wilson_stencil(U, mcrit + 0.01).to_sparse()
    init = [_vecs(4, L * L, 2, 5)]
    sb = [synth.gaussian_field((L * L * 2,), synth.rng_for(129))]
    H, vecs = normal.adaptive_setup(D, (L, L), [(4, 4)], [4], init, sb, nu0=10, ncyc=2)
    A = H.ops[0]
    rq = [np.linalg.norm(A.apply(v.reshape(-1))) / np.linalg.norm(v) for v in vecs[0]]
    rq0 = [np.linalg.norm(A.apply(v.reshape(-1))) / np.linalg.norm(v) for v in init[0]]
    assert max(rq) < 0.5 * min(rq0)
    Hr = normal.build(D, (L, L), init, [(4, 4)], sb)
    chi = np.zeros(L * L * 2, dtype=np.complex128)
    chi[0] = 1.0
    b = D.conj().T @ chi
    it_a, it_r = normal.mgcg(H, b, 1e-10)[1], normal.mgcg(Hr, b, 1e-10)[1]
    assert it_a.converged and it_r.converged
    assert it_a.iters < 0.8 * it_r.iters


def test_fine_applications_per_mgcg_iteration():
    """Per MG-CG iteration the fine operator is applied 5 times: once in the
    outer CG, twice by the pre-smoother, once to form the residual before
    post-smoothing and once by the post-smoother (the paper counts 6: it runs
    the post-smoother as two full steps whose last residual goes unused)."""
    D, H, _ = _hier(16, [(4, 4)], [4])
    A = H.ops[0]
    b = synth.gaussian_field((A.n,), synth.rng_for(130))
    A.napply = 0
    _, info = normal.mgcg(H, b, 1e-10)
    # + one recomputed residual at the convergence check and one for rel_res
    assert info.converged and A.napply == 5 * info.iters + 2


def _hier_sa(L, blocks, nvec, sa, m=0.05, seed=0):
    D = _D(L, m, seed)
    dims = [(L, L)]
    vecs, sb = [], []
    for l, (b, nv) in enumerate(zip(blocks, nvec)):
        V = dims[-1][0] * dims[-1][1]
        dof = 2 if l == 0 else nvec[l - 1]
        vecs.append(_vecs(nv, V, dof, seed * 10 + l))
        sb.append(synth.gaussian_field((V * dof,), synth.rng_for(122, seed, l)))
        dims.append((dims[-1][0] // b[0], dims[-1][1] // b[1]))
    return D, normal.build(D, (L, L), vecs, blocks, sb, sa=sa), vecs, sb


def test_normal_operator_is_a_box_stencil():
    """D^dag D couples x to x + (a, b) with |a|, |b| <= 1 only (the straight
    double hop cancels), all nine couplings nonzero."""
    L = 8
    D = _D(L, 0.05)
    A = abs((D.conj().T @ D).toarray()).reshape(L * L, 2, L * L, 2).sum((1, 3))
    x, y = np.arange(L * L) % L, np.arange(L * L) // L
    dx = np.minimum((x[:, None] - x[None, :]) % L, (x[None, :] - x[:, None]) % L)
    dy = np.minimum((y[:, None] - y[None, :]) % L, (y[None, :] - y[:, None]) % L)
    box = (dx <= 1) & (dy <= 1)
    assert A[~box].max() < 1e-14 and A[box].min() > 0.0


def test_power_estimate_bounds_the_largest_eigenvalue():
    D = _D(16, 0.05)
    A = normal.CountingOp((D.conj().T @ D).tocsr())
    lmax = np.linalg.eigvalsh(A.M.toarray()).max()
    v0 = synth.gaussian_field((A.n,), synth.rng_for(131))
    est = [normal.power_lmax(A, v0, k) for k in (0, 5, 20, 80)]
    assert all(e <= lmax * (1 + 1e-12) for e in est)
    assert est[0] < est[1] <= est[2] <= est[3] and est[3] > 0.95 * lmax


def test_smoothed_prolongator_support_and_coarse_reach():
    """P = (1 - omega A) P_tent.  With r = 1 the spin projectors of a
    straight double hop multiply to zero, so D^dag D couples a site only to
    its 3 x 3 box: a smoothed column of block j lives on the block widened by
    one site on every side (corners included), and for 4 x 4 blocks the
    Galerkin operator still couples only neighbouring blocks (diagonal ones
    included): a 9-point box stencil on the coarse lattice."""
    L, b = 32, 4
    D, H, vecs, sb = _hier_sa(L, [(b, b)], [4], sa=4.0 / 3.0)
    A = H.ops[0]
    Pt = normal.block_prolongator(vecs[0], (L, L), (b, b))
    om = H.sa_omegas[0]
    assert om > 0 and abs(om - (4.0 / 3.0) / normal.power_lmax(A, sb[0], 20)) < 1e-15
    P = H.Ps[0]
    assert abs(P - (Pt - om * (A.M @ Pt))).max() < 1e-14
    x = np.arange(L * L) % L
    y = np.arange(L * L) // L
    Lc = L // b
    for j in (0, 5, Lc * Lc - 1):
        jx, jy = j % Lc, j // Lc
        col = np.abs(P[:, j * 4].toarray().reshape(L * L, 2)).sum(1)
        ox, oy = (x - jx * b) % L, (y - jy * b) % L          # offsets from the block's corner
        ex = np.where(ox < b, 0, np.minimum(ox - (b - 1), L - ox))
        ey = np.where(oy < b, 0, np.minimum(oy - (b - 1), L - oy))
        inside = (ex <= 1) & (ey <= 1)
        assert col[~inside].max() == 0.0 and col[inside].min() > 0.0
    C = abs(H.ops[1].M.toarray()).reshape(Lc * Lc, 4, Lc * Lc, 4).sum((1, 3))
    cx, cy = np.arange(Lc * Lc) % Lc, np.arange(Lc * Lc) // Lc
    ddx = np.minimum((cx[:, None] - cx[None, :]) % Lc, (cx[None, :] - cx[:, None]) % Lc)
    ddy = np.minimum((cy[:, None] - cy[None, :]) % Lc, (cy[None, :] - cy[:, None]) % Lc)
    near = (ddx <= 1) & (ddy <= 1)
    assert C[~near].max() == 0.0 and C[near].min() > 0.0


def test_smoothed_vcycle_equals_operator_formula():
    """Eq. (3) holds for any P, the smoothed one included."""
    D, H, _, _ = _hier_sa(8, [(4, 4)], [3], sa=4.0 / 3.0)
    V = _vcycle_matrix(H)
    A = H.ops[0].M.toarray()
    P = H.Ps[0].toarray()
    Ac = H.ops[1].M.toarray()
    assert np.abs(Ac - P.conj().T @ A @ P).max() < 1e-12 * np.abs(Ac).max()
    t0, t1 = H.taus[0]
    I = np.eye(A.shape[0])
    R = (t0 + t1) * I - t0 * t1 * A
    ref = R + R.conj().T - R @ A @ R.conj().T + (I - R @ A) @ P @ np.linalg.inv(Ac) @ P.conj().T @ (I - A @ R.conj().T)
    assert np.abs(V - ref).max() < 1e-10 * np.abs(ref).max()
