"""Critical mass from the spectrum of D (oracle; test infrastructure only).

The mass gap is m_hat = m - m_crit (numerical-test section), with m_crit the
mass at which the smallest real part of the spectrum of D(m) reaches zero:
m_crit = -min_k Re lambda_k(D(m = 0)).  The spectrum shifts exactly with m,
so one eigenvalue computation at m = 0 fixes m_crit.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mg import Stencil


def leftmost_eigenvalues(A0: Stencil, k: int = 4, shifts=(-0.05,)) -> np.ndarray:
    """Eigenvalues of A0 with the smallest real parts.

    Dense for up to 4096 unknowns; beyond that ARPACK on (A0 - s)^-1 (sparse
    LU) at real shifts s left of the spectrum, pooling the eigenvalues
    nearest to each shift.  The leftmost eigenvalues of the Wilson operator
    lie close to the real axis, so the ones nearest a shift on the real axis
    left of the spectrum include them."""
    N = A0.V * A0.dof
    if N <= 4096:
        ev = np.linalg.eigvals(A0.to_sparse().toarray())
        return ev[np.argsort(ev.real)][:k]
    M = A0.to_sparse().tocsc()
    pool = []
    for s in shifts:
        lu = spla.splu((M - s * sp.identity(N, format="csc")).tocsc())
        op = spla.LinearOperator(M.shape, matvec=lu.solve, dtype=np.complex128)
        mu = spla.eigs(op, k=k, which="LM", return_eigenvectors=False, tol=1e-6,
                       ncv=max(4 * k, 40), maxiter=100000)
        pool.append(1.0 / mu + s)
    ev = np.concatenate(pool)
    return ev[np.argsort(ev.real)][:k]


def critical_mass(A0: Stencil) -> tuple[float, complex]:
    """(m_crit, leftmost eigenvalue of D(0))."""
    ev = leftmost_eigenvalues(A0)
    return float(-ev[0].real), complex(ev[0])
