"""Pins of oracle functions that the other oracle tests do not reach.

* the stored workload table is reproduced by the script that wrote it;
* the critical-mass estimate (both eigensolver branches) against the
  closed-form free-field spectrum and against dense eigenvalues of the
  matrix built entry by entry from the paper's definition of D;
* the GCR of the coarsest level and of the K-cycle against minimal-residual
  least-squares problems solved directly (GCR's defining property), and the
  converged K-cycle against a two-grid cycle with an exact coarse solve;
* the exact coarsest solve of the V-cycle against the Galerkin property of an
  exact coarse-grid correction.
"""
import json

import numpy as np
import pytest

import synth
from oracle import dirac, make_workloads, mg, spectrum


def _field(L1, L2, beta=6.0, sweeps=30, seed=0):
    th = synth.u1_heatbath(L1, L2, beta, sweeps, synth.rng_for(97, seed, L1, L2))
    return dirac.u1_field(th)


def _vecs(n, V, dof, seed):
    return np.stack([synth.gaussian_field((V, dof), synth.rng_for(98, seed, k)) for k in range(n)])


# ---------------------------------------------------------------------------
# the workload table
# ---------------------------------------------------------------------------

def test_workload_table_is_reproduced():
    """Regenerate the 32^2 entry: plaquette and charge identical, m_crit to
    the eigensolver tolerance (the other entries: `--check` of the script)."""
    with open(make_workloads.OUT) as f:
        table = json.load(f)
    w = [w for w in make_workloads.WORKLOADS if w[0] == "schwinger_32_b6"][0]
    name, e = make_workloads.entry(w)
    assert make_workloads.compare(table[name], e) == []
    assert table[name]["plaquette"] == e["plaquette"] and table[name]["Q"] == e["Q"]


# ---------------------------------------------------------------------------
# critical mass
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,dense_max", [((16, 16), 4096), ((24, 24), 0), ((4, 4, 4, 4), 4096),
                                            ((4, 4, 2, 4), 0)])
def test_free_field_critical_mass_is_zero(dims, dense_max):
    """At U = 1 the leftmost eigenvalue of D(0) is lambda(p = 0) = 0 (closed
    form), so m_crit = 0; the four leftmost eigenvalues are the closed-form
    ones.  dense_max = 0 forces the shift-invert branch."""
    nd = len(dims)
    nc = 1 if nd == 2 else 3
    U = np.zeros((nd,) + tuple(reversed(dims)) + (nc, nc), dtype=np.complex128)
    U[...] = np.eye(nc)
    A0 = mg.wilson_stencil(U, 0.0)
    mcrit, lam = spectrum.critical_mass(A0, dense_max=dense_max)
    assert abs(mcrit) < 1e-9 and abs(lam) < 1e-9
    ev = spectrum.leftmost_eigenvalues(A0, k=4, dense_max=dense_max)
    ref = dirac.free_field_eigenvalues(dims, 0.0, nc)
    ref = np.sort_complex(ref[np.argsort(ref.real, kind="stable")][:4])
    assert np.abs(np.sort(ev.real) - np.sort(ref.real)).max() < 1e-8


@pytest.mark.parametrize("L,beta,seed", [(16, 6.0, 0), (16, 3.0, 1), (12, 10.0, 2)])
def test_shift_invert_matches_dense_eigenvalues(L, beta, seed):
    """Both branches of the eigensolver against numpy's eigenvalues of the
    dense matrix built entry by entry from the definition of D."""
    U = _field(L, L, beta=beta, sweeps=60, seed=seed)
    ev_ref = np.linalg.eigvals(dirac.dense_D(U, 0.0))
    ev_ref = ev_ref[np.argsort(ev_ref.real)]
    A0 = mg.wilson_stencil(U, 0.0)
    for dense_max in (4096, 0):
        ev = spectrum.leftmost_eigenvalues(A0, k=4, dense_max=dense_max)
        # the four leftmost (real parts in order; conjugate pairs tie) ...
        assert np.abs(np.sort(ev.real) - ev_ref.real[:4]).max() < 1e-9
        # ... and each one an eigenvalue of the dense spectrum
        for e in ev:
            assert np.abs(ev_ref - e).min() < 1e-8
    mcrit, _ = spectrum.critical_mass(A0)
    assert abs(mcrit + ev_ref[0].real) < 1e-9
    # the spectrum shifts exactly with the mass
    mcrit2, _ = spectrum.critical_mass(mg.wilson_stencil(U, 0.25))
    assert abs(mcrit2 - (mcrit - 0.25)) < 1e-9


@pytest.mark.slow
def test_default_shift_invert_branch_above_dense_limit():
    """46^2 (4232 unknowns) takes the shift-invert branch by default; it must
    find the leftmost eigenvalue of the dense spectrum."""
    L = 46
    U = _field(L, L, beta=6.0, sweeps=60, seed=5)
    A0 = mg.wilson_stencil(U, 0.0)
    assert A0.V * A0.dof > 4096
    mcrit, lam = spectrum.critical_mass(A0)
    ev_ref = np.linalg.eigvals(A0.to_sparse().toarray())
    assert abs(mcrit + ev_ref.real.min()) < 1e-9
    assert np.abs(ev_ref - lam).min() < 1e-8
    # the leftmost mode of this field is a complex pair: a single real shift
    # with four eigenvalues finds other modes first
    assert abs(lam.imag) > 0.05


# ---------------------------------------------------------------------------
# GCR (coarsest level, K-cycle) and the exact coarsest solve
# ---------------------------------------------------------------------------

def _min_res_reference(A, b, M, steps, restart):
    """Iterates of the minimal-residual method over the preconditioned search
    space, solved as least-squares problems: within a restart cycle started
    at x0, z_j = M(b - A x_{j-1}) and x_j = x0 + argmin_{y in span(z_1..z_j)}
    ||b - A (x0 + y)||."""
    x = np.zeros_like(b)
    x0 = x.copy()
    Z = []
    for it in range(steps):
        if it % restart == 0:
            x0, Z = x.copy(), []
        Z.append(M(b - A.apply(x)).reshape(-1))
        Zm = np.stack(Z, axis=1)
        AZ = np.stack([A.apply(z.reshape(b.shape)).reshape(-1) for z in Z], axis=1)
        y = np.linalg.lstsq(AZ, (b - A.apply(x0)).reshape(-1), rcond=None)[0]
        x = x0 + (Zm @ y).reshape(b.shape)
    return x


@pytest.mark.parametrize("precond,steps,restart", [(False, 6, 6), (False, 9, 4), (True, 5, 5), (True, 7, 3)])
def test_gcr_is_minimal_residual(precond, steps, restart):
    """gcr_coarse after k steps equals the minimal-residual iterate over the
    span of its search directions (restarted), with and without a fixed
    preconditioner."""
    U = _field(8, 8, seed=3)
    A = mg.wilson_stencil(U, 0.08)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(99, 1))
    if precond:
        rng = synth.rng_for(99, 2)
        N = A.V * A.dof
        Mm = np.eye(N) + 0.3 * synth.gaussian_field((N, N), rng) / np.sqrt(N)
        M = lambda r: (Mm @ r.reshape(-1)).reshape(r.shape)  # noqa: E731
    else:
        M = lambda r: r.copy()  # noqa: E731
    x = mg.gcr_coarse(A, b, 0.0, steps, restart, precond=M if precond else None)
    ref = _min_res_reference(A, b, M, steps, restart)
    assert mg.norm(x - ref) < 1e-10 * mg.norm(ref)


def test_gcr_stop_rule():
    """tol >= 1: x = 0 satisfies the stopping rule before any step."""
    U = _field(8, 8, seed=3)
    A = mg.wilson_stencil(U, 0.08)
    b = synth.gaussian_field((A.V, 2), synth.rng_for(99, 3))
    assert mg.norm(mg.gcr_coarse(A, b, 1.0, 10, 10)) == 0.0
    x = mg.gcr_coarse(A, b, 1e-3, 500, 500)
    assert mg.norm(b - A.apply(x)) <= 1e-3 * mg.norm(b)


def test_converged_kcycle_equals_exact_two_grid():
    """A K-cycle whose intermediate level is solved to 1e-13 equals the
    two-grid cycle with that level solved exactly (dense), to ~1e-11."""
    U = _field(16, 16, seed=4)
    A = mg.wilson_stencil(U, 0.05)
    v0 = _vecs(4, A.V, 2, 1)
    A1 = mg.galerkin(A, mg.build_prolongator(v0, A.dims, (4, 4)))
    v1 = _vecs(3, A1.V, A1.dof, 2)
    p3 = mg.MGParams(blocks=[(4, 4), (2, 2)], nvec=[4, 3], kcycle_tol=1e-13, kcycle_maxiter=200)
    H3 = mg.build_hierarchy(A, [v0, v1], p3)
    p2 = mg.MGParams(blocks=[(4, 4)], nvec=[4])
    H2 = mg.Hierarchy(H3.ops[:2], H3.Ps[:1], p2)
    assert H2.ops[1].V * H2.ops[1].dof <= p2.coarse_dense_max
    b = synth.gaussian_field((A.V, 2), synth.rng_for(99, 4))
    xk = mg.vcycle(H3, 0, b)
    x2 = mg.vcycle(H2, 0, b)
    assert mg.norm(xk - x2) < 1e-11 * mg.norm(x2)
    # and the two-grid cycle's coarse solve really is exact: with no
    # post-smoothing the correction leaves a P^dag-orthogonal residual
    p0 = mg.MGParams(blocks=[(4, 4)], nvec=[4], nu_post=0)
    H0 = mg.Hierarchy(H3.ops[:2], H3.Ps[:1], p0)
    x0 = mg.vcycle(H0, 0, b)
    assert mg.norm(H3.Ps[0].restrict(b - A.apply(x0))) < 1e-12 * mg.norm(b)


def test_kcycle_one_step_is_minimal_residual_multiple():
    """One K-cycle step on the intermediate level: x1 = alpha z with
    z = V_1(b1) and alpha = <A z, b1>/<A z, A z> (the minimal-residual
    multiple of the preconditioned direction)."""
    U = _field(16, 16, seed=5)
    A = mg.wilson_stencil(U, 0.05)
    v0 = _vecs(4, A.V, 2, 3)
    A1 = mg.galerkin(A, mg.build_prolongator(v0, A.dims, (4, 4)))
    v1 = _vecs(2, A1.V, A1.dof, 4)
    p = mg.MGParams(blocks=[(4, 4), (2, 2)], nvec=[4, 2], kcycle_tol=0.0, kcycle_maxiter=1)
    H = mg.build_hierarchy(A, [v0, v1], p)
    b1 = synth.gaussian_field((H.ops[1].V, H.ops[1].dof), synth.rng_for(99, 5))
    z = mg.vcycle(H, 1, b1)
    w = H.ops[1].apply(z)
    alpha = mg.vdot(w, b1) / mg.vdot(w, w).real
    x1 = mg.gcr_coarse(H.ops[1], b1, 0.0, 1, 1, precond=lambda r: mg.vcycle(H, 1, r))
    assert mg.norm(x1 - alpha * z) < 1e-13 * mg.norm(x1)


def test_dense_coarsest_solve_is_exact():
    """The exact coarsest solve returns A^-1 b (against numpy's solve of the
    sparse triple product P^dag D P); a hierarchy marks a level exact by its
    size, and the adaptive setup by the size of the finished level."""
    U = _field(8, 8, seed=6)
    A = mg.wilson_stencil(U, 0.05)
    P = mg.build_prolongator(_vecs(4, A.V, 2, 5), A.dims, (4, 4))
    Ac = mg.galerkin(A, P)
    b = synth.gaussian_field((Ac.V, Ac.dof), synth.rng_for(99, 6))
    x = mg.coarsest_solve(Ac, b, mg.MGParams(blocks=[(4, 4)], nvec=[4]), exact=True)
    Ps = P.to_sparse()
    M = (Ps.conj().T @ A.to_sparse() @ Ps).toarray()
    ref = np.linalg.solve(M, b.ravel())
    assert mg.norm(x.ravel() - ref) < 1e-12 * mg.norm(ref)
    # a level not marked exact is solved by GCR to coarse_tol
    x2 = mg.coarsest_solve(Ac, b, mg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_tol=1e-2), exact=False)
    assert mg.norm(b - Ac.apply(x2)) <= 1e-2 * mg.norm(b)
    assert mg.norm(x2.ravel() - ref) > 1e-9 * mg.norm(ref)
    p = mg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_dense_max=Ac.V * Ac.dof)
    assert mg.Hierarchy([A, Ac], [P], p).exact == [False, True]
    p.coarse_dense_max -= 1
    assert mg.Hierarchy([A, Ac], [P], p).exact == [False, False]


def test_block_jacobi_coarsest_gcr():
    """The block-Jacobi preconditioned coarsest GCR: on an operator without
    hops (block diagonal) one step is its exact inverse, site by site (numpy
    solves of the non-symmetric blocks, so a transposed or conjugated block
    fails); the first step on a Galerkin operator is the residual minimiser
    along A M b with M the inverse diagonal blocks; to a tight tolerance it
    returns the dense solution, not that of A M."""
    rng = np.random.default_rng(5)
    V, n = 16, 6
    diag = 3.0 * np.eye(n) + rng.standard_normal((V, n, n)) + 1j * rng.standard_normal((V, n, n))
    Ab = mg.Stencil((4, 4), n, diag, np.zeros((4, V, n, n), complex))
    b = rng.standard_normal((V, n)) + 1j * rng.standard_normal((V, n))
    pj = mg.MGParams(blocks=[(4, 4)], nvec=[3], coarse_tol=1e-14, coarse_maxiter=1, coarse_jacobi=True)
    x = mg.coarsest_solve(Ab, b, pj, exact=False)
    ref = np.stack([np.linalg.solve(diag[s], b[s]) for s in range(V)])
    assert mg.norm(x - ref) < 1e-13 * mg.norm(ref)
    x_plain = mg.coarsest_solve(Ab, b, mg.MGParams(blocks=[(4, 4)], nvec=[3], coarse_tol=1e-14, coarse_maxiter=1),
                                exact=False)
    assert mg.norm(x_plain - ref) > 1e-2 * mg.norm(ref)
    # a Galerkin operator with hops
    U = _field(8, 8, seed=6)
    A = mg.wilson_stencil(U, 0.05)
    P = mg.build_prolongator(_vecs(4, A.V, 2, 5), A.dims, (4, 4))
    Ac = mg.galerkin(A, P)
    bc = synth.gaussian_field((Ac.V, Ac.dof), synth.rng_for(99, 7))
    Mb = np.stack([np.linalg.solve(Ac.diag[s], bc[s]) for s in range(Ac.V)])
    w = Ac.apply(Mb)
    alpha = mg.vdot(w, bc) / mg.vdot(w, w).real
    x1 = mg.coarsest_solve(Ac, bc, mg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_tol=0.0, coarse_maxiter=1,
                                                coarse_jacobi=True), exact=False)
    assert mg.norm(x1 - alpha * Mb) < 1e-13 * mg.norm(x1)
    xt = mg.coarsest_solve(Ac, bc, mg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_tol=1e-12, coarse_maxiter=400,
                                                coarse_restart=16, coarse_jacobi=True), exact=False)
    xd = mg.dense_solve(Ac, bc)
    assert mg.norm(xt - xd) < 1e-9 * mg.norm(xd)


def test_even_odd_coarsest_solve():
    """The even-odd reduced coarsest GCR: its Schur operator equals
    1 - T_eo T_oe taken from the sparse matrix of T = A M (M the inverse
    diagonal blocks, so T_ee = T_oo = 1); to a tight tolerance it returns the
    dense solution; the residual of a loose solve is at most coarse_tol |b|
    and lies on the even sites only."""
    import scipy.sparse as sp
    U = _field(16, 16, seed=8)
    A = mg.wilson_stencil(U, 0.05)
    P = mg.build_prolongator(_vecs(4, A.V, 2, 7), A.dims, (2, 2))
    Ac = mg.galerkin(A, P)                                   # 8 x 8 coarse sites, 8 dof
    n = Ac.dof
    Minv = np.linalg.inv(Ac.diag)
    T = (Ac.to_sparse() @ sp.block_diag(list(Minv), format="csr")).toarray()
    x1 = np.arange(Ac.V) % Ac.dims[0]
    x2 = np.arange(Ac.V) // Ac.dims[0]
    ev = np.where((x1 + x2) % 2 == 0)[0]
    od = np.where((x1 + x2) % 2 == 1)[0]
    ie = (ev[:, None] * n + np.arange(n)).ravel()
    io = (od[:, None] * n + np.arange(n)).ravel()
    assert np.allclose(T[np.ix_(ie, ie)], np.eye(len(ie)), atol=1e-13)
    Sd = np.eye(len(ie)) - T[np.ix_(ie, io)] @ T[np.ix_(io, ie)]
    b = synth.gaussian_field((Ac.V, n), synth.rng_for(99, 8))
    # the operator the solver builds, reached through one GCR step from x = 0
    seen = {}
    orig = mg.gcr_coarse

    def spy(op, rhs, *a, **k):
        seen["op"] = op
        return orig(op, rhs, *a, **k)
    mg.gcr_coarse = spy
    try:
        p = mg.MGParams(blocks=[(2, 2)], nvec=[4], coarse_tol=1e-12, coarse_maxiter=500, coarse_restart=32,
                        coarse_jacobi=True, coarse_eo=True)
        xt = mg.coarsest_solve(Ac, b, p, exact=False)
    finally:
        mg.gcr_coarse = orig
    v = synth.gaussian_field((len(ev), n), synth.rng_for(99, 9))
    assert np.linalg.norm(seen["op"].apply(v).ravel() - Sd @ v.ravel()) < 1e-12 * np.linalg.norm(v)
    xd = mg.dense_solve(Ac, b)
    assert mg.norm(xt - xd) < 1e-9 * mg.norm(xd)
    p.coarse_tol = 0.2
    xl = mg.coarsest_solve(Ac, b, p, exact=False)
    r = b - Ac.apply(xl)
    assert mg.norm(r) <= 0.2 * mg.norm(b) * (1 + 1e-12)
    assert mg.norm(r[od]) < 1e-12 * mg.norm(b)
