"""Adaptive multigrid for D psi = chi (oracle; test infrastructure only).

Plain FP64 NumPy.  Every routine follows the paper's definitions in the
order they are stated; nothing is blocked, fused or reordered.

Operators are nearest-neighbour block stencils on a periodic lattice:

  (A f)(x) = diag(x) f(x) + sum_{dir} hop_dir(x) f(x + dir),

with dir = 2*mu for +mu and 2*mu + 1 for -mu.  The fine Wilson-Dirac
operator is one such stencil (see `wilson_stencil`), and so is every
Galerkin coarse operator P^dagger A P (Eq. (2)), because P is block local.

Coarse degrees of freedom are chirally split: for each block S_j and
chirality chi = +, - the near-null vectors restricted to the block and
projected on that chirality are orthonormalised, and the coarse dof index is
t = chi * N_v + k (chirality major), so the coarse gamma_5 is
diag(+1_{N_v}, -1_{N_v}).  On the fine lattice the chirality of a spin-colour
component is fixed by gamma_5 being diagonal: the first half of the
components per site is chi = +.  This holds for the 2d Pauli basis
(gamma_5 = sigma_3), the 4d chiral basis and every coarse level.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .lattice import gammas, site_coords, site_index


def vdot(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm(a: np.ndarray) -> float:
    return float(np.linalg.norm(a.ravel()))


# ----------------------------------------------------------------------------
# Block stencil operator
# ----------------------------------------------------------------------------

def neighbour_table(dims) -> np.ndarray:
    """nbr[dir, x] = index of x + dir, dir = 2 mu (+mu), 2 mu + 1 (-mu)."""
    nd = len(dims)
    c = site_coords(dims)
    out = np.empty((2 * nd, c.shape[0]), dtype=np.int64)
    for mu in range(nd):
        e = np.zeros(nd, dtype=np.int64)
        e[mu] = 1
        out[2 * mu] = site_index(c + e, dims)
        out[2 * mu + 1] = site_index(c - e, dims)
    return out


@dataclass
class Stencil:
    """A = diag + sum_dir hop_dir shift_dir on a periodic lattice of `dims`."""
    dims: tuple
    dof: int
    diag: np.ndarray            # (V, dof, dof)
    hop: np.ndarray             # (2 nd, V, dof, dof)
    napply: int = 0             # number of single-vector applications (cost counter)
    nbr: np.ndarray = field(default=None, repr=False)
    _lu: tuple = field(default=None, repr=False)   # dense LU factors (coarsest-level solves)

    def __post_init__(self):
        if self.nbr is None:
            self.nbr = neighbour_table(self.dims)

    @property
    def nd(self) -> int:
        return len(self.dims)

    @property
    def V(self) -> int:
        return int(np.prod(self.dims))

    def apply(self, f: np.ndarray) -> np.ndarray:
        """A f for f of shape (V, dof)."""
        self.napply += 1
        out = np.einsum("xab,xb->xa", self.diag, f)
        for d in range(2 * self.nd):
            out += np.einsum("xab,xb->xa", self.hop[d], f[self.nbr[d]])
        return out

    def apply_dagger(self, f: np.ndarray) -> np.ndarray:
        """A^dagger f: the adjoint of every block, scattered back along its hop."""
        self.napply += 1
        out = np.einsum("xba,xb->xa", np.conj(self.diag), f)
        for d in range(2 * self.nd):
            contrib = np.einsum("xba,xb->xa", np.conj(self.hop[d]), f)
            np.add.at(out, self.nbr[d], contrib)
        return out

    def to_sparse(self) -> sp.csr_matrix:
        """The operator as a sparse matrix, row/column index = site * dof + component."""
        V, n = self.V, self.dof
        x = np.arange(V)[:, None, None]
        a = np.arange(n)[None, :, None]
        b = np.arange(n)[None, None, :]
        row = np.broadcast_to(x * n + a, (V, n, n))
        rows = [row.ravel()]
        cols = [np.broadcast_to(x * n + b, (V, n, n)).ravel()]
        vals = [self.diag.ravel()]
        for d in range(2 * self.nd):
            rows.append(row.ravel())
            cols.append(np.broadcast_to(self.nbr[d][:, None, None] * n + b, (V, n, n)).ravel())
            vals.append(self.hop[d].ravel())
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(V * n, V * n))

    def shifted(self, dm: float, mass_matrix: np.ndarray) -> "Stencil":
        """Copy with diag + dm * mass_matrix (per-site (dof, dof) blocks)."""
        return Stencil(self.dims, self.dof, self.diag + dm * mass_matrix, self.hop.copy(),
                       nbr=self.nbr)


def wilson_stencil(U: np.ndarray, m: float) -> Stencil:
    """The Wilson-Dirac operator (definition after Eq. (1)) as a block stencil.

    diag = (d + m) 1;  hop_{+mu}(x) = -1/2 (1 - gamma_mu) (x) U_mu(x);
    hop_{-mu}(x) = -1/2 (1 + gamma_mu) (x) U_mu(x - mu)^dagger.
    Spin-colour component index = spin * nc + colour.
    """
    nd = U.shape[0]
    dims = tuple(reversed(U.shape[1:1 + nd]))
    nc = U.shape[-1]
    ns = 2 if nd == 2 else 4
    dof = ns * nc
    V = int(np.prod(dims))
    g = gammas(nd)
    eye = np.eye(ns)
    Uf = U.reshape(nd, V, nc, nc)
    nbr = neighbour_table(dims)
    diag = np.broadcast_to((nd + m) * np.eye(dof, dtype=np.complex128), (V, dof, dof)).copy()
    hop = np.zeros((2 * nd, V, dof, dof), dtype=np.complex128)
    for mu in range(nd):
        hop[2 * mu] = -0.5 * np.einsum("st,xab->xsatb", eye - g[mu], Uf[mu]).reshape(V, dof, dof)
        U_back = np.conj(np.swapaxes(Uf[mu][nbr[2 * mu + 1]], -1, -2))
        hop[2 * mu + 1] = -0.5 * np.einsum("st,xab->xsatb", eye + g[mu], U_back).reshape(V, dof, dof)
    return Stencil(dims, dof, diag, hop, nbr=nbr)


def gamma5_diag(dof: int) -> np.ndarray:
    """Diagonal of gamma_5 per site in the chirality-major component order."""
    h = dof // 2
    return np.concatenate([np.ones(h), -np.ones(h)])


# ----------------------------------------------------------------------------
# Geometric blocks and the chirally split prolongator (Eq. (5) and the
# construction of v_{sj} that follows it)
# ----------------------------------------------------------------------------

class RankError(RuntimeError):
    """A block's projected near-null vectors are linearly dependent."""


@dataclass
class Prolongator:
    fine_dims: tuple
    block: tuple
    dof: int                    # fine components per site
    nvec: int                   # N_v (coarse dof = 2 N_v)
    Q: np.ndarray               # (V, dof, 2 N_v): rows of P at every fine site
    blk: np.ndarray             # (V,) coarse site of every fine site

    @property
    def coarse_dims(self) -> tuple:
        return tuple(L // b for L, b in zip(self.fine_dims, self.block))

    @property
    def nc(self) -> int:
        return 2 * self.nvec

    @property
    def Vc(self) -> int:
        return int(np.prod(self.coarse_dims))

    def restrict(self, r: np.ndarray) -> np.ndarray:
        """r_hat(j)[t] = sum_{x in S_j} sum_a conj(P(x)[a, t]) r(x)[a]   (P^dagger r)."""
        out = np.zeros((self.Vc, self.nc), dtype=np.complex128)
        np.add.at(out, self.blk, np.einsum("xat,xa->xt", np.conj(self.Q), r))
        return out

    def prolong(self, e: np.ndarray) -> np.ndarray:
        """(P e)(x)[a] = sum_t P(x)[a, t] e(block(x))[t]."""
        return np.einsum("xat,xt->xa", self.Q, e[self.blk])

    def to_sparse(self) -> sp.csr_matrix:
        """P as a sparse (V*dof) x (Vc*2N_v) matrix."""
        V, n, nc = self.Q.shape
        rows = np.broadcast_to(np.arange(V)[:, None, None] * n + np.arange(n)[None, :, None], (V, n, nc))
        cols = np.broadcast_to(self.blk[:, None, None] * nc + np.arange(nc)[None, None, :], (V, n, nc))
        return sp.csr_matrix((self.Q.ravel(), (rows.ravel(), cols.ravel())), shape=(V * n, self.Vc * nc))


def block_map(dims, block):
    """Coarse site of every fine site, and the fine-site coordinates."""
    if any(L % b for L, b in zip(dims, block)):
        raise ValueError("lattice extents must be multiples of the block extents")
    c = site_coords(dims)
    cdims = tuple(L // b for L, b in zip(dims, block))
    blk = site_index(c // np.asarray(block), cdims)
    return blk, c


def orthonormalise_block(W: np.ndarray, rank_tol: float = 1e-10) -> np.ndarray:
    """Modified Gram-Schmidt applied twice, in column order, R_kk > 0.

    The paper makes each new block vector orthogonal to the previous ones and
    normalises it to 1; applying the sweep twice keeps the result orthonormal
    to rounding.  A column whose remainder falls below rank_tol times its
    original norm is reported as a rank error rather than dropped.
    """
    W = W.astype(np.complex128).copy()
    n = W.shape[1]
    for k in range(n):
        w0 = np.linalg.norm(W[:, k])
        w = W[:, k]
        for _ in range(2):
            for j in range(k):
                w = w - np.vdot(W[:, j], w) * W[:, j]
        nrm = np.linalg.norm(w)
        if not (nrm > rank_tol * w0) or w0 == 0.0:
            raise RankError(f"block vector {k} is linearly dependent")
        W[:, k] = w / nrm
    return W


def build_prolongator(vecs: np.ndarray, dims, block) -> Prolongator:
    """P from near-null vectors vecs (N_v, V, dof), chirally split per block.

    For block S_j and chirality chi, the vectors (Pi_chi v_k)|_{S_j} are
    orthonormalised (k = 1..N_v in order) and become the columns
    t = chi N_v + k of P restricted to that block.
    """
    nv, V, dof = vecs.shape
    h = dof // 2
    blk, _ = block_map(dims, block)
    Vc = int(blk.max()) + 1
    Q = np.zeros((V, dof, 2 * nv), dtype=np.complex128)
    for j in range(Vc):
        sites = np.nonzero(blk == j)[0]
        for chi in range(2):
            comp = slice(chi * h, (chi + 1) * h)
            W = vecs[:, sites, comp].reshape(nv, -1).T        # (bs*h, N_v)
            Wo = orthonormalise_block(W)
            Q[sites, comp, chi * nv:(chi + 1) * nv] = Wo.reshape(len(sites), h, nv)
    return Prolongator(tuple(dims), tuple(block), dof, nv, Q, blk)


# ----------------------------------------------------------------------------
# Galerkin coarse operator, Eq. (2), applied to D:  D_hat = P^dagger D P
# ----------------------------------------------------------------------------

def galerkin(A: Stencil, P: Prolongator) -> Stencil:
    """D_hat = P^dagger A P written as a coarse block stencil.

    Each fine hop x -> x + dir lands in the coarse block coupling block(x)
    to block(x + dir).  A hop that leaves the block through its face (x_mu
    on the last layer of the block for +mu, on the first layer for -mu) is
    a coarse hop in direction dir; every other hop, and the diagonal, stays
    inside the block and goes to the coarse diagonal.  Classifying by the
    face crossed (not by which block is reached) keeps coarse extents of 1
    or 2 correct.
    """
    dims, block = A.dims, P.block
    nd = len(dims)
    c = site_coords(dims)
    Vc, nc = P.Vc, P.nc
    Qc = np.conj(P.Q)
    diag = np.zeros((Vc, nc, nc), dtype=np.complex128)
    hop = np.zeros((2 * nd, Vc, nc, nc), dtype=np.complex128)
    np.add.at(diag, P.blk, np.einsum("xat,xab,xbs->xts", Qc, A.diag, P.Q))
    for mu in range(nd):
        for sgn, d in ((+1, 2 * mu), (-1, 2 * mu + 1)):
            contrib = np.einsum("xat,xab,xbs->xts", Qc, A.hop[d], P.Q[A.nbr[d]])
            face = block[mu] - 1 if sgn > 0 else 0
            cross = (c[:, mu] % block[mu]) == face
            np.add.at(hop[d], P.blk[cross], contrib[cross])
            np.add.at(diag, P.blk[~cross], contrib[~cross])
    return Stencil(P.coarse_dims, nc, diag, hop)


def galerkin_mass_matrix(M: np.ndarray, P: Prolongator) -> np.ndarray:
    """P^dagger M P for a block-diagonal (per site) matrix M: the derivative
    of the coarse operator with respect to the fine mass."""
    out = np.zeros((P.Vc, P.nc, P.nc), dtype=np.complex128)
    np.add.at(out, P.blk, np.einsum("xat,xab,xbs->xts", np.conj(P.Q), M, P.Q))
    return out


# ----------------------------------------------------------------------------
# Smoother, Krylov solvers and the V-cycle
# ----------------------------------------------------------------------------

def mr(A: Stencil, b: np.ndarray, nu: int, omega: float, x0: np.ndarray | None = None):
    """Under-relaxed minimal residual (the paper's MR smoother, run on D).

    Starting from x (0 by default) with r = b - A x, repeat nu times:
    p = A r; alpha = <p, r>/<p, p>; x += omega alpha r; r -= omega alpha p.
    Returns (x, r), r being the recursively updated residual.
    """
    if x0 is None:
        x = np.zeros_like(b, dtype=np.complex128)
        r = b.astype(np.complex128).copy()
    else:
        x = x0.astype(np.complex128).copy()
        r = b - A.apply(x)
    for _ in range(nu):
        p = A.apply(r)
        pp = vdot(p, p).real
        if pp == 0.0:
            break
        alpha = omega * vdot(p, r) / pp
        x = x + alpha * r
        r = r - alpha * p
    return x, r


@dataclass
class SolveInfo:
    iters: int = 0
    converged: bool = False
    true_rel_res: float = np.inf
    history: list = field(default_factory=list)


def fgcr(A: Stencil, b: np.ndarray, precond, tol: float, maxiter: int, restart: int,
         x0: np.ndarray | None = None):
    """Flexible GCR (Eisenstat, Elman and Schultz's GCR with a varying preconditioner).

    Each iteration: z = M(r); w = A z; orthogonalise w against the stored
    w_j (coefficients beta_j = <w_j, w>/<w_j, w_j>, all taken from the same
    w) and apply the same combination to z; alpha = <w, r>/<w, w>;
    x += alpha z; r -= alpha w.  After `restart` directions, or when the
    recursive residual meets the tolerance, the true residual b - A x
    replaces r and the directions are dropped.  Converged means
    ||b - A x|| <= tol ||b|| for the true residual.
    """
    bnorm = norm(b)
    x = np.zeros_like(b, dtype=np.complex128) if x0 is None else x0.astype(np.complex128).copy()
    r = b.astype(np.complex128) - (A.apply(x) if x0 is not None else 0)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.true_rel_res = True, 0.0
        return x, info
    Z, W, WW = [], [], []
    while True:
        rn = norm(r)
        info.history.append(rn / bnorm)
        if rn <= tol * bnorm:
            r = b - A.apply(x)
            info.true_rel_res = norm(r) / bnorm
            if info.true_rel_res <= tol:
                info.converged = True
                break
            Z, W, WW = [], [], []
        if info.iters >= maxiter:
            break
        z = precond(r)
        w = A.apply(z)
        betas = [vdot(W[j], w) / WW[j] for j in range(len(W))]
        for j, beta in enumerate(betas):
            w = w - beta * W[j]
            z = z - beta * Z[j]
        ww = vdot(w, w).real
        alpha = vdot(w, r) / ww
        x = x + alpha * z
        r = r - alpha * w
        Z.append(z); W.append(w); WW.append(ww)
        info.iters += 1
        if len(W) == restart:
            r = b - A.apply(x)
            Z, W, WW = [], [], []
    if not info.converged:
        info.true_rel_res = norm(b - A.apply(x)) / bnorm
    return x, info


def cgnr(A: Stencil, b: np.ndarray, tol: float, maxiter: int):
    """CG on the normal equations D^dagger D x = D^dagger b (the paper's CG baseline).

    r = b; s = A^dag r; p = s; gamma = ||s||^2; each iteration
    q = A p; alpha = gamma/||q||^2; x += alpha p; r -= alpha q;
    s = A^dag r; gamma' = ||s||^2; p = s + (gamma'/gamma) p.
    Stops on ||r||/||b|| of the original system.  One A and one A^dag per iteration.
    """
    bnorm = norm(b)
    x = np.zeros_like(b, dtype=np.complex128)
    r = b.astype(np.complex128).copy()
    s = A.apply_dagger(r)
    p = s.copy()
    gamma = vdot(s, s).real
    info = SolveInfo()
    while norm(r) > tol * bnorm and info.iters < maxiter:
        q = A.apply(p)
        alpha = gamma / vdot(q, q).real
        x = x + alpha * p
        r = r - alpha * q
        s = A.apply_dagger(r)
        gnew = vdot(s, s).real
        p = s + (gnew / gamma) * p
        gamma = gnew
        info.iters += 1
    info.true_rel_res = norm(b - A.apply(x)) / bnorm
    info.converged = info.true_rel_res <= tol
    return x, info


@dataclass
class MGParams:
    blocks: list                      # block extents per coarsening
    nvec: list                        # N_v per coarsening
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8
    coarse_dense_max: int = 4096      # coarsest level solved exactly (dense LU) up to this many unknowns
    coarse_tol: float = 0.1           # coarsest-level GCR relative tolerance (larger coarsest levels)
    coarse_maxiter: int = 64
    coarse_restart: int = 16
    outer_restart: int = 16
    smoother: object = None           # callable(A, b, nu, omega) -> (x, r); MR when None
    kcycle_tol: float = None          # intermediate levels: GCR to this tolerance (K-cycle); None: V-cycle
    kcycle_maxiter: int = 8
    coarse_jacobi: bool = False       # coarsest GCR preconditioned by the inverse diagonal blocks (dof <= 48)
    coarse_eo: bool = False           # with coarse_jacobi on 2d levels of even extents: even-odd reduced GCR


@dataclass
class Hierarchy:
    ops: list                         # Stencil per level, finest first
    Ps: list                          # Prolongator per coarsening
    params: MGParams
    mass_mats: list = None            # d(op)/dm per level (per-site blocks)
    exact: list = None                # per level: solved exactly when it is the coarsest level of a cycle

    def __post_init__(self):
        if self.exact is None:
            self.exact = [A.V * A.dof <= self.params.coarse_dense_max for A in self.ops]

    @property
    def nlevels(self) -> int:
        return len(self.ops)


def gcr_coarse(A: Stencil, b: np.ndarray, tol: float, maxiter: int, restart: int, precond=None) -> np.ndarray:
    """Approximate level solve: GCR from x = 0 (flexible when a preconditioner is given).

    Used for a coarsest level too large for the exact solve, and with a
    preconditioner M for the K-cycle's intermediate levels.  GCR minimises
    the residual over the span of the search directions; iteration it:
    stop if ||r|| <= tol ||b|| (recursive residual; checked before the first
    step too, so x = 0 is returned when tol >= 1); at the start of every
    restart cycle after the first, r = b - A x and the stored directions are
    dropped; then z = r (or z = M(r)), w = A z, w and z are orthogonalised
    against the stored directions (classical Gram-Schmidt coefficients
    <w_j, w>/<w_j, w_j>), alpha = <w, r>/<w, w>, x += alpha z, r -= alpha w.
    At most maxiter iterations.
    """
    x = np.zeros_like(b, dtype=np.complex128)
    r = b.astype(np.complex128).copy()
    bb = vdot(b, b).real
    done = vdot(r, r).real <= tol * tol * bb
    Z, W, WW = [], [], []
    for it in range(maxiter):
        if done:
            break
        if it % restart == 0 and it > 0:
            r = b - A.apply(x)
            Z, W, WW = [], [], []
        z = r.copy() if precond is None else precond(r)
        w = A.apply(z)
        betas = [(vdot(W[j], w) / WW[j]) if WW[j] > 0 else 0.0 for j in range(len(W))]
        for j, beta in enumerate(betas):
            w = w - beta * W[j]
            z = z - beta * Z[j]
        ww = vdot(w, w).real
        alpha = vdot(w, r) / ww if ww > 0 else 0.0
        x = x + alpha * z
        r = r - alpha * w
        Z.append(z); W.append(w); WW.append(ww)
        done = vdot(r, r).real <= tol * tol * bb
    return x


def dense_solve(A: Stencil, b: np.ndarray) -> np.ndarray:
    """x = A^-1 b by LU with partial pivoting of the dense matrix of A (the
    factors are kept on the operator for later solves)."""
    if getattr(A, "_lu", None) is None:
        A._lu = sla.lu_factor(A.to_sparse().toarray())
    return sla.lu_solve(A._lu, b.reshape(-1)).reshape(b.shape)


def coarsest_solve(A: Stencil, b: np.ndarray, p: MGParams, exact: bool) -> np.ndarray:
    """Solve on the coarsest level of a cycle.  The paper solves its coarsest
    lattice exactly; that is done here for a level marked exact (one of at
    most coarse_dense_max unknowns when all its near-null vectors are in
    place).  Other levels are solved approximately by GCR to coarse_tol (see
    gcr_coarse; the outer Krylov method is flexible)."""
    if exact:
        return dense_solve(A, b)
    precond = None
    if p.coarse_jacobi and A.dof <= 48:
        if p.coarse_eo and A.nd == 2 and A.dims[0] % 2 == 0 and A.dims[1] % 2 == 0:
            return eo_jacobi_solve(A, b, p)
        precond = lambda r: block_jacobi(A, r)
    return gcr_coarse(A, b, p.coarse_tol, p.coarse_maxiter, p.coarse_restart, precond=precond)


class _SchurOp:
    """v_e -> v_e - T_eo T_oe v_e for the unit-diagonal operator T = A M."""

    def __init__(self, hops, even, odd, V, dof):
        self.hops, self.even, self.odd, self.V, self.dof = hops, even, odd, V, dof
        self.napply = 0

    def embed(self, v, sites):
        f = np.zeros((self.V, self.dof), dtype=np.complex128)
        f[sites] = v
        return f

    def apply(self, v):
        self.napply += 1
        t = self.hops(self.embed(v, self.even))[self.odd]            # T_oe v
        return v - self.hops(self.embed(t, self.odd))[self.even]     # v - T_eo t


def eo_jacobi_solve(A: Stencil, b: np.ndarray, p: MGParams) -> np.ndarray:
    """Coarsest GCR on the even sites of the block-Jacobi preconditioned
    system: with M the inverse diagonal blocks, T = A M has a unit diagonal;
    split by site parity, T y = b is (1 - T_eo T_oe) y_e = b_e - T_eo b_o and
    y_o = b_o - T_oe y_e, and x = M y.  GCR stops when the even residual
    (the whole residual: the odd part is zero) is at most coarse_tol |b|."""
    Minv = np.linalg.inv(A.diag)
    Thop = [A.hop[d] @ Minv[A.nbr[d]] for d in range(2 * A.nd)]      # T(x, x + d) = A_d(x) M(x + d)

    def hops(f):                                                    # (T - 1) f
        out = np.zeros_like(f)
        for d in range(2 * A.nd):
            out += np.einsum("xab,xb->xa", Thop[d], f[A.nbr[d]])
        return out

    x1 = np.arange(A.V) % A.dims[0]
    x2 = np.arange(A.V) // A.dims[0]
    even = np.where((x1 + x2) % 2 == 0)[0]
    odd = np.where((x1 + x2) % 2 == 1)[0]
    S = _SchurOp(hops, even, odd, A.V, A.dof)
    bp = b[even] - hops(S.embed(b[odd], odd))[even]
    nb, nbp = norm(b), norm(bp)
    if p.coarse_tol >= 1.0 or nbp == 0.0:
        ye = np.zeros_like(bp)
    else:
        ye = gcr_coarse(S, bp, p.coarse_tol * nb / nbp, p.coarse_maxiter, p.coarse_restart)
    A.napply += S.napply
    yo = b[odd] - hops(S.embed(ye, even))[odd]
    y = np.zeros((A.V, A.dof), dtype=np.complex128)
    y[even], y[odd] = ye, yo
    return np.einsum("xab,xb->xa", Minv, y)


def block_jacobi(A: Stencil, r: np.ndarray) -> np.ndarray:
    """z(x) = diag(x)^-1 r(x): each site's diagonal block of A inverted and
    applied to r (the block-Jacobi preconditioner of the coarsest GCR; the
    paper's coarsest solve is exact, this only speeds up its approximation)."""
    return np.linalg.solve(A.diag, r[..., None])[..., 0]


def vcycle(H: Hierarchy, level: int, b: np.ndarray) -> np.ndarray:
    """One V-cycle on `level` (the five steps listed before Eq. (3), applied to D).

    1. pre-relax: x from nu_pre MR steps on A x = b (r its residual);
    2. restrict the residual r_hat = P^dagger r;
    3. e_hat = V^{(l+1)} r_hat (approximate solve on the coarsest level);
    4. correct x += P e_hat;
    5. post-relax on the new residual: x += MR_{nu_post}(b - A x).
    Step 5 is read as x <- x + R(b - A x): the printed 'x = R(b - Ax)'
    drops the existing iterate.
    """
    p = H.params
    A = H.ops[level]
    if level == H.nlevels - 1:
        return coarsest_solve(A, b, p, H.exact[level])
    relax = mr if p.smoother is None else p.smoother
    P = H.Ps[level]
    x, r = relax(A, b, p.nu_pre, p.omega)
    rc = P.restrict(r)
    if p.kcycle_tol is not None and level + 1 < H.nlevels - 1:
        # K-cycle: the intermediate level is solved by flexible GCR
        # preconditioned by its own cycle
        ec = gcr_coarse(H.ops[level + 1], rc, p.kcycle_tol, p.kcycle_maxiter, p.kcycle_maxiter,
                        precond=lambda rr: vcycle(H, level + 1, rr))
    else:
        ec = vcycle(H, level + 1, rc)
    x = x + P.prolong(ec)
    r = b - A.apply(x)
    x = x + relax(A, r, p.nu_post, p.omega)[0]
    return x


def build_hierarchy(A0: Stencil, vecs: list, params: MGParams) -> Hierarchy:
    """Levels from given near-null vectors: P_l from vecs[l] (N_v, V_l, dof_l),
    A_{l+1} = P_l^dagger A_l P_l."""
    ops, Ps = [A0], []
    mass = [np.broadcast_to(np.eye(A0.dof, dtype=np.complex128), (A0.V, A0.dof, A0.dof))]
    for lvl, v in enumerate(vecs):
        P = build_prolongator(v, ops[-1].dims, params.blocks[lvl])
        Ps.append(P)
        ops.append(galerkin(ops[-1], P))
        mass.append(galerkin_mass_matrix(mass[-1], P))
    return Hierarchy(ops, Ps, params, mass)


def with_mass(H: Hierarchy, dm: float) -> Hierarchy:
    """Reuse the setup at another mass (the paper reuses the null vectors of the
    lightest mass for heavier ones): every level shifts by dm times P^dag...P."""
    ops = [A.shifted(dm, M) for A, M in zip(H.ops, H.mass_mats)]
    return Hierarchy(ops, H.Ps, H.params, H.mass_mats, H.exact)


def mg_solve(H: Hierarchy, b: np.ndarray, tol: float = 1e-10, maxiter: int = 500):
    """FGCR on the finest level preconditioned by one V-cycle per iteration."""
    return fgcr(H.ops[0], b, lambda r: vcycle(H, 0, r), tol, maxiter, H.params.outer_restart)


# ----------------------------------------------------------------------------
# Adaptive setup (text from Eq. (4) through the recursion remark after Eq. (5))
# ----------------------------------------------------------------------------

def relax_homogeneous(A: Stencil, v: np.ndarray, nu: int, omega: float) -> np.ndarray:
    """nu MR steps on A v = 0 starting at v (the first adaptive pass, Eq. (4) read for D)."""
    return mr(A, np.zeros_like(v), nu, omega, x0=v)[0]


def adaptive_setup(A0: Stencil, params: MGParams, init: list, nu0: int = 20, ncyc: int = 2):
    """Adaptive construction of the near-null vectors, level by level.

    For coarsening l with operator A_l and random starting vectors init[l]
    (N_v, V_l, dof_l):
      (i)  v_1 = init[l][0] relaxed by nu0 MR steps on A_l v = 0; build P_l
           from {v_1} and A_{l+1} = P_l^dag A_l P_l;
      (ii) for k = 2..N_v: e = init[l][k-1]; apply ncyc sweeps of the
           two-level error propagation e <- e - V(A_l e) (A_{l+1} solved as
           the coarsest level: exactly if the finished level, with all N_v
           vectors, has at most coarse_dense_max unknowns, else by GCR);
           v_k = e/||e||; rebuild P_l and A_{l+1}.
    With l fixed, the procedure recurses on A_{l+1} (the method is recursive).
    Returns (hierarchy, vecs) with vecs[l] of shape (N_v, V_l, dof_l).
    """
    ops = [A0]
    all_vecs = []
    for lvl in range(len(params.blocks)):
        A = ops[-1]
        nv = params.nvec[lvl]
        vecs = [relax_homogeneous(A, init[lvl][0], nu0, params.omega)]
        for k in range(1, nv + 1):
            P = build_prolongator(np.stack(vecs), A.dims, params.blocks[lvl])
            Ac = galerkin(A, P)
            if k == nv:
                break
            exact_c = Ac.V * 2 * nv <= params.coarse_dense_max
            H2 = Hierarchy([A, Ac], [P], params, exact=[False, exact_c])
            e = init[lvl][k].astype(np.complex128).copy()
            for _ in range(ncyc):
                e = e - vcycle(H2, 0, A.apply(e))
            vecs.append(e / norm(e))
        all_vecs.append(np.stack(vecs))
        ops.append(Ac)
    return build_hierarchy(A0, all_vecs, params), all_vecs
