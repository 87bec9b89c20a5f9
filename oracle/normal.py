"""Multigrid for the normal equations A = D^dagger D, the paper's own variant
(oracle; test infrastructure only).

Plain FP64 NumPy/SciPy; every operator is a scipy.sparse matrix built from
its definition, so nothing is blocked or fused:

* A_0 = D^dagger D (D the Wilson-Dirac operator, definition after Eq. (1));
* P_l: the M near-null vectors restricted to each block S_j of the level's
  lattice and orthonormalised there (Eq. (5) and the text after it; one
  coarse degree of freedom per vector, no chiral split), optionally smoothed
  by one damped Richardson step, P_l = (1 - omega_l A_l) P_l^tent ("smoothed
  aggregation", adaptive-method section), with omega_l = f / lambda_l and
  lambda_l the Rayleigh quotient of A_l after a fixed number of power steps;
  A_{l+1} = P_l^dagger A_l P_l (Eq. (2), Hermitian positive definite);
* the smoother: two under-relaxed minimal-residual steps (omega = 0.8) whose
  step lengths are computed once from a given vector and then frozen, so the
  relaxation is a fixed polynomial in A with R = R^dagger (numerical-test
  section);
* the V-cycle: the five steps before Eq. (3) with R^dagger before and R
  after the coarse-grid correction, the coarsest level solved exactly; the
  resulting operator is Hermitian (Eq. (3), read with "- R A R^dagger");
* conjugate gradients preconditioned by one V-cycle per iteration
  (MG-CG), and plain CG on the same system, both stopping on the relative
  residual of A x = b.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mg


def vdot(a, b) -> complex:
    return complex(np.vdot(np.ravel(a), np.ravel(b)))


def norm(a) -> float:
    return float(np.linalg.norm(np.ravel(a)))


class CountingOp:
    """A sparse Hermitian operator with a count of its applications."""

    def __init__(self, M: sp.spmatrix, fine_D_per_apply: int = 0):
        self.M = M.tocsr()
        self.n = M.shape[0]
        self.napply = 0
        self.fine_D_per_apply = fine_D_per_apply   # D / D^dag applications one application stands for

    def apply(self, x: np.ndarray) -> np.ndarray:
        self.napply += 1
        return self.M @ x


def block_prolongator(vecs: np.ndarray, dims, block) -> sp.csr_matrix:
    """P (V*dof) x (Vc*M) from vecs (M, V, dof): on each block S_j the M
    vectors restricted to S_j (all components together) are orthonormalised
    by modified Gram-Schmidt applied twice, in vector order, and become the
    M columns of P belonging to coarse site j."""
    M, V, dof = vecs.shape
    blk, _ = mg.block_map(dims, block)
    Vc = int(blk.max()) + 1
    rows, cols, vals = [], [], []
    for j in range(Vc):
        sites = np.nonzero(blk == j)[0]
        W = vecs[:, sites, :].reshape(M, -1).T            # (bs*dof, M)
        Q = mg.orthonormalise_block(W)
        idx = (sites[:, None] * dof + np.arange(dof)[None, :]).ravel()
        for k in range(M):
            rows.append(idx)
            cols.append(np.full(idx.size, j * M + k))
            vals.append(Q[:, k])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(V * dof, Vc * M))


def power_lmax(A: CountingOp, v0: np.ndarray, kpow: int) -> float:
    """<p, A p> / <p, p> after kpow steps p <- A p / |A p| from v0: an
    estimate of A's largest eigenvalue from below."""
    p = v0.astype(np.complex128) / norm(v0)
    for _ in range(kpow):
        q = A.apply(p)
        p = q / norm(q)
    return vdot(p, A.apply(p)).real


def smoothed_prolongator(A: CountingOp, Pt: sp.spmatrix, f: float, v0: np.ndarray, kpow: int):
    """(P, omega): P = (1 - omega A) Pt with omega = f / power_lmax(A, v0, kpow);
    f = 0 returns Pt itself."""
    if f == 0.0:
        return Pt.tocsr(), 0.0
    omega = f / power_lmax(A, v0, kpow)
    return (Pt - omega * (A.M @ Pt)).tocsr(), omega


def frozen_steps(A: CountingOp, b: np.ndarray, omega: float) -> tuple[float, float]:
    """Step lengths tau_i = omega alpha_i of two MR steps on A x = b from x = 0,
    alpha = <A r, r> / <A r, A r> (real for Hermitian A; the real part is
    taken)."""
    taus = []
    r = b.astype(np.complex128).copy()
    for _ in range(2):
        p = A.apply(r)
        alpha = vdot(p, r).real / vdot(p, p).real
        taus.append(omega * alpha)
        r = r - omega * alpha * p
    return taus[0], taus[1]


@dataclass
class NormalHierarchy:
    ops: list                        # CountingOp per level, finest first
    Ps: list                         # sparse prolongators
    dims: list                       # lattice extents per level
    taus: list                       # frozen smoother steps per level (all but the coarsest)
    coarse_lu: object = None         # factors of the coarsest operator
    sa_omegas: list = field(default_factory=list)   # Richardson damping of each P (0: unsmoothed)

    @property
    def nlevels(self) -> int:
        return len(self.ops)


def smooth(A: CountingOp, b: np.ndarray, taus) -> tuple[np.ndarray, np.ndarray]:
    """x = R b from x = 0 and its residual b - A x: the two frozen steps
    x += tau_i r, r -= tau_i A r (two applications of A)."""
    x = np.zeros_like(b)
    r = b.copy()
    for t in taus:
        x = x + t * r
        r = r - t * A.apply(r)
    return x, r


def smooth_add(A: CountingOp, r: np.ndarray, taus) -> np.ndarray:
    """R r (the same polynomial, without its final residual): one application of A."""
    t0, t1 = taus
    return (t0 + t1) * r - (t0 * t1) * A.apply(r)


def vcycle(H: NormalHierarchy, level: int, b: np.ndarray) -> np.ndarray:
    """One V-cycle (the five steps before Eq. (3)) on level `level`."""
    A = H.ops[level]
    if level == H.nlevels - 1:
        return H.coarse_lu.solve(b)
    P = H.Ps[level]
    x, r = smooth(A, b, H.taus[level])                 # 1. x = R^dag b (R = R^dag)
    e = vcycle(H, level + 1, P.conj().T @ r)           # 2.-3. restrict the residual, cycle below
    x = x + P @ e                                      # 4. coarse-grid correction
    return x + smooth_add(A, b - A.apply(x), H.taus[level])   # 5. x += R (b - A x)


def build(D: sp.spmatrix, dims, vecs: list, blocks: list, smoother_b: list, omega: float = 0.8,
          sa: float = 0.0, kpow: int = 20) -> NormalHierarchy:
    """Hierarchy from given near-null vectors vecs[l] (M, V_l, dof_l) and the
    vectors smoother_b[l] the frozen step lengths (and the power estimate of
    the smoothing damping, sa = f > 0) are computed from."""
    ops = [CountingOp((D.conj().T @ D).tocsr(), fine_D_per_apply=2)]
    Ps, ds, taus, oms = [], [tuple(dims)], [], []
    for l, (v, blk) in enumerate(zip(vecs, blocks)):
        P, om = smoothed_prolongator(ops[-1], block_prolongator(v, ds[-1], blk), sa, smoother_b[l], kpow)
        Ps.append(P)
        oms.append(om)
        ops.append(CountingOp((P.conj().T @ ops[-1].M @ P).tocsr()))
        ds.append(tuple(L // b for L, b in zip(ds[-1], blk)))
    for l in range(len(ops) - 1):
        taus.append(frozen_steps(ops[l], smoother_b[l], omega))
        ops[l].napply = 0
    H = NormalHierarchy(ops, Ps, ds, taus, sa_omegas=oms)
    H.coarse_lu = spla.splu(ops[-1].M.tocsc())
    return H


def relax_homogeneous(A: CountingOp, v: np.ndarray, nu: int, omega: float) -> np.ndarray:
    """nu under-relaxed MR steps on A v = 0 from v (the first adaptive pass, Eq. (4))."""
    v = v.astype(np.complex128).copy()
    r = -A.apply(v)
    for _ in range(nu):
        p = A.apply(r)
        alpha = omega * vdot(p, r) / vdot(p, p).real
        v = v + alpha * r
        r = r - alpha * p
    return v


class _CGCoarse:
    """Coarse solve of the set-up cycles by plain CG to a relative residual
    (used where the coarse level is too large to factor)."""

    def __init__(self, A: CountingOp, tol: float, maxiter: int):
        self.A, self.tol, self.maxiter = A, tol, maxiter

    def solve(self, b):
        return pcg(self.A, b, None, self.tol, self.maxiter)[0]


def adaptive_setup(D: sp.spmatrix, dims, blocks: list, nvec: list, init: list, smoother_b: list,
                   nu0=20, ncyc=2, omega: float = 0.8, sa: float = 0.0, kpow: int = 20,
                   setup_dense_max=None, setup_coarse_tol: float = 1e-6, setup_coarse_maxiter: int = 20000):
    """Adaptive construction for A = D^dag D, level by level (text from Eq. (4)
    to the recursion remark after Eq. (5)): vector 1 of coarsening l is
    init[l][0] after nu0 MR relaxations on A_l v = 0; vector k > 1 is
    init[l][k-1] after ncyc sweeps of e <- e - V(A_l e) with the two-level
    cycle of the vectors so far, normalised.  nu0 and ncyc are numbers or one
    number per coarsening.  The prolongators of the set-up cycles are
    smoothed like the final ones (sa).  The coarse level of a set-up cycle is
    solved exactly (factored) when setup_dense_max is None or it has at most
    setup_dense_max unknowns, else by CG to setup_coarse_tol.
    Returns (hierarchy, vecs)."""
    nl = len(blocks)
    nu0 = list(nu0) if np.ndim(nu0) else [nu0] * nl
    ncyc = list(ncyc) if np.ndim(ncyc) else [ncyc] * nl
    A0 = (D.conj().T @ D).tocsr()
    ops = [CountingOp(A0, fine_D_per_apply=2)]
    ds = [tuple(dims)]
    all_vecs = []
    for l, blk in enumerate(blocks):
        A = ops[-1]
        shape = init[l][0].shape                        # (V_l, dof_l)
        taus = frozen_steps(A, smoother_b[l], omega)
        vecs = [relax_homogeneous(A, init[l][0].reshape(-1), nu0[l], omega)]
        for k in range(1, nvec[l]):
            Pt = block_prolongator(np.stack([v.reshape(shape) for v in vecs]), ds[-1], blk)
            P, _ = smoothed_prolongator(A, Pt, sa, smoother_b[l], kpow)
            Ac = CountingOp((P.conj().T @ A.M @ P).tocsr())
            exact = setup_dense_max is None or Ac.n <= setup_dense_max
            cs = spla.splu(Ac.M.tocsc()) if exact else _CGCoarse(Ac, setup_coarse_tol, setup_coarse_maxiter)
            H2 = NormalHierarchy([A, Ac], [P], [ds[-1]], [taus], cs)
            e = init[l][k].reshape(-1).astype(np.complex128).copy()
            for _ in range(ncyc[l]):
                e = e - vcycle(H2, 0, A.apply(e))
            vecs.append(e / norm(e))
        all_vecs.append(np.stack([v.reshape(shape) for v in vecs]))
        P, _ = smoothed_prolongator(A, block_prolongator(all_vecs[-1], ds[-1], blk), sa, smoother_b[l], kpow)
        ops.append(CountingOp((P.conj().T @ A.M @ P).tocsr()))
        ds.append(tuple(L // b for L, b in zip(ds[-1], blk)))
    H = build(D, dims, all_vecs, blocks, smoother_b, omega, sa, kpow)
    return H, all_vecs


@dataclass
class CGInfo:
    iters: int = 0
    converged: bool = False
    rel_res: float = np.inf           # |b - A x| / |b|, recomputed
    history: list = field(default_factory=list)


def pcg(A: CountingOp, b: np.ndarray, precond, tol: float, maxiter: int):
    """Conjugate gradients on A x = b preconditioned by `precond` (identity:
    plain CG).  z = M r; rho = <r, z>; p = z + (rho / rho_old) p; q = A p;
    alpha = rho / <p, q>; x += alpha p; r -= alpha q.  Stops when the
    recursive residual is below tol |b| and the recomputed one confirms it."""
    bn = norm(b)
    x = np.zeros_like(b, dtype=np.complex128)
    r = b.astype(np.complex128).copy()
    info = CGInfo()
    p = None
    rho_old = None
    while info.iters < maxiter:
        if norm(r) <= tol * bn:
            rt = b - A.apply(x)
            if norm(rt) <= tol * bn:
                info.converged = True
                break
            r = rt
            p = None
        z = r.copy() if precond is None else precond(r)
        rho = vdot(r, z).real
        p = z.copy() if p is None else z + (rho / rho_old) * p
        q = A.apply(p)
        alpha = rho / vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rho_old = rho
        info.iters += 1
        info.history.append(norm(r) / bn)
    info.rel_res = norm(b - A.apply(x)) / bn
    info.converged = info.rel_res <= tol
    return x, info


def mgcg(H: NormalHierarchy, b: np.ndarray, tol: float, maxiter: int = 1000):
    """CG preconditioned by one V-cycle per iteration."""
    return pcg(H.ops[0], b, lambda r: vcycle(H, 0, r), tol, maxiter)


def with_mass(D_of_mass, H: NormalHierarchy, vecs: list, blocks: list, smoother_b: list, dims,
              omega: float = 0.8, sa: float = 0.0, kpow: int = 20) -> NormalHierarchy:
    """The hierarchy of the same near-null vectors at another mass: every
    Galerkin product rebuilt from D(m) (A(m) = D(m)^dag D(m) is not a shift of
    A(m0)), the step lengths recomputed."""
    return build(D_of_mass, dims, vecs, blocks, smoother_b, omega, sa, kpow)
