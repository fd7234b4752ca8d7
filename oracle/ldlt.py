"""Plain dense LDL^T with 1x1 pivots (test infrastructure only).

Algorithm 1 factors every diagonal block as A_i = L_i D_i L_i^T and the Schur
complement as S = L_s D_s L_s^T (section 4.2). The blocks of the MPOPF KKT are
quasi-definite (positive definite Hessian part, negative definite dual part),
so an LDL^T with 1x1 pivots exists in any symmetric order.

The paper leaves the pivot perturbation to the sparse solver (section 2.1 lists
scaling, matching and pivoting; section 2.3 the inertia). The reading used
here and in the library (static pivoting): pivot k is perturbed when
|d_k| <= tau_k with tau_k = eps * |a_kk| (the original diagonal entry of the
matrix being factored), or tau_k = eps * max|A| when a_kk = 0. The pivot keeps
its computed sign (the expected sign s_k, +1 primal / -1 dual or Schur, when
d_k = 0) and takes the magnitude tau_k. The threshold is invariant under
symmetric diagonal scaling. Inertia is counted from the computed pivots
before perturbation, so a wrong-sign pivot is reported, not hidden.

Inertia (section 2.3): the triple (n+, n-, n0) of eigenvalue signs; for
A = L D L^T it equals the sign count of D (Sylvester's law of inertia).
"""
from __future__ import annotations

import numpy as np


def ldlt(A, signs=None, eps: float = 1e-20, return_raw: bool = False):
    """Right-looking LDL^T of the symmetric matrix A in its given order.

    Returns (L, d, n_perturbed) with L unit lower triangular and A = L diag(d) L^T
    (exactly, up to rounding, when nothing was perturbed); with return_raw also
    the computed pivots before perturbation (whose signs give the inertia)."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    amax = np.max(np.abs(A)) if n else 0.0
    diag0 = np.abs(np.diag(A)).copy()
    L = np.eye(n)
    d = np.empty(n)
    raw = np.empty(n)
    npert = 0
    for k in range(n):
        dk = A[k, k]
        raw[k] = dk
        tau = eps * (diag0[k] if diag0[k] > 0 else amax)
        if abs(dk) <= tau:
            s = np.sign(dk) if dk != 0 else (signs[k] if signs is not None else 1.0)
            dk = s * tau
            npert += 1
            if dk == 0.0:
                raise ZeroDivisionError(f"zero pivot at {k}")
        d[k] = dk
        col = A[k + 1:, k]
        l = col / dk
        L[k + 1:, k] = l
        # trailing update A22 -= l * d_k * l^T
        A[k + 1:, k + 1:] -= np.outer(l * dk, l)
    if return_raw:
        return L, d, npert, raw
    return L, d, npert


def ldlt_solve(L, d, b):
    """Solve (L diag(d) L^T) x = b for b of shape [n] or [n, k]."""
    import scipy.linalg as sl
    y = sl.solve_triangular(L, b, lower=True, unit_diagonal=True)
    y = (y.T / d).T
    return sl.solve_triangular(L.T, y, lower=False, unit_diagonal=True)


def inertia_from_d(d):
    d = np.asarray(d)
    return int(np.sum(d > 0)), int(np.sum(d < 0)), int(np.sum(d == 0))


def inertia_eig(A, rtol: float = 0.0):
    """Inertia from the eigenvalues of the dense symmetric A (brute force)."""
    w = np.linalg.eigvalsh(np.asarray(A, dtype=np.float64))
    thr = rtol * (np.max(np.abs(w)) if w.size else 0.0)
    return int(np.sum(w > thr)), int(np.sum(w < -thr)), int(np.sum(np.abs(w) <= thr))
