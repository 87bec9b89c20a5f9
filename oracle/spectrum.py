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


def leftmost_eigenvalues(A0: Stencil, k: int = 4, shifts=(-0.05, -0.05 + 0.1j, -0.05 + 0.2j), nev: int = 16,
                         dense_max: int = 4096) -> np.ndarray:
    """Eigenvalues of A0 with the smallest real parts.

    Dense for up to dense_max unknowns.  Beyond that, ARPACK on (A0 - s)^-1
    (sparse LU) finds the nev eigenvalues nearest to each shift s, and the
    pool is sorted by real part.  The shifts sit left of the spectrum, on and
    above the real axis: the leftmost modes of a rough gauge field can be
    complex pairs whose imaginary part puts several eigenvalues with larger
    real parts nearer to a single real shift (the spectrum is symmetric under
    conjugation, because D is gamma_5-Hermitian, so shifts below the axis
    would find the conjugates)."""
    N = A0.V * A0.dof
    if N <= dense_max:
        ev = np.linalg.eigvals(A0.to_sparse().toarray())
        return ev[np.argsort(ev.real)][:k]
    M = A0.to_sparse().tocsc().astype(np.complex128)
    pool = []
    for s in shifts:
        lu = spla.splu((M - s * sp.identity(N, format="csc", dtype=np.complex128)).tocsc())
        op = spla.LinearOperator(M.shape, matvec=lu.solve, dtype=np.complex128)
        mu = spla.eigs(op, k=max(k, nev), which="LM", return_eigenvectors=False, tol=1e-10,
                       ncv=max(4 * max(k, nev), 40), maxiter=100000)
        # an eigenvalue found again from another shift is the same one; a
        # repeated eigenvalue within one shift's set is a multiplicity
        matched = set()
        for lam in 1.0 / mu + s:
            j = next((j for j, q in enumerate(pool) if j not in matched and abs(q - lam) <= 1e-8), None)
            if j is None:
                pool.append(lam)
                j = len(pool) - 1
            matched.add(j)
    ev = np.array(pool)
    return ev[np.argsort(ev.real)][:k]


def critical_mass(A0: Stencil, dense_max: int = 4096) -> tuple[float, complex]:
    """(m_crit, leftmost eigenvalue of D(0))."""
    ev = leftmost_eigenvalues(A0, dense_max=dense_max)
    return float(-ev[0].real), complex(ev[0])
