"""Krylov solvers of the oracle: CG, Jacobi-PCG, flexible CG, iterative refinement.

Test infrastructure only (see the package docstring).

Notation follows the paper's Alg. 1 with the roles renamed: the paper's
search direction ``x`` is ``p`` here, its solution ``y`` is ``x``, and its
Jacobian ``J`` is ``-A`` (CG is unchanged by flipping the sign of both the
operator and the residual). The loop is textbook Hestenes-Stiefel CG.

Readings where the paper is silent:

* the stopping test is relative and unsquared, ``||r_{k+1}|| <= tol*||b||``, on
  the recursively updated residual (Alg. 1 tests an absolute threshold on the
  squared norm of the previous residual);
* the initial guess is zero unless one is given;
* flexible CG takes the Polak-Ribiere beta of Golub and Ye (1999),
  ``beta = z_{k+1}.(r_{k+1} - r_k) / (z_k.r_k)``, with no restarts;
* iterative refinement computes residuals in FP64 and solves each correction
  with the same CG carried out in FP32 (NumPy float32 arithmetic).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    rel_res: float                      # recursive residual / ||b|| at exit
    history: list = field(default_factory=list)   # ||r_k|| / ||b|| for k = 0..iters
    status: str = "ok"                  # "ok" | "max_iter" | "breakdown"
    outer: int = 0                      # refinement steps (refinement only)


def cg(A, b, x0=None, tol=1e-6, max_iter=10000, dtype=np.float64, callback=None):
    """Conjugate gradient on ``A x = b`` (Alg. 1).

    ``A`` is anything with ``A @ v``; all vectors and scalars are held in
    ``dtype``. ``callback(k, x, r, p)`` sees the state after each iteration.
    """
    return pcg(A, b, None, x0=x0, tol=tol, max_iter=max_iter, dtype=dtype, callback=callback)


def pcg(A, b, M, x0=None, tol=1e-6, max_iter=10000, dtype=np.float64, callback=None):
    """Preconditioned CG; ``M(r)`` returns ``z``. ``M=None`` is plain CG (z = r)."""
    b = np.asarray(b, dtype=dtype)
    A_ = A.astype(dtype) if hasattr(A, "astype") else A
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=dtype).copy()
    r = b - A_ @ x if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    if nb == 0:
        return SolveResult(x=x, iters=0, converged=True, rel_res=0.0, history=[0.0])
    z = r if M is None else np.asarray(M(r), dtype=dtype)
    rho = r @ z
    p = z.copy()
    hist = [float(np.linalg.norm(r) / nb)]
    if hist[0] <= tol:
        return SolveResult(x=x, iters=0, converged=True, rel_res=hist[0], history=hist)
    for k in range(max_iter):
        q = A_ @ p
        pq = p @ q
        if not (pq > 0) or not np.isfinite(pq):
            return SolveResult(x=x, iters=k, converged=False, rel_res=hist[-1],
                               history=hist, status="breakdown")
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        rn = np.linalg.norm(r)
        hist.append(float(rn / nb))
        if callback is not None:
            callback(k, x, r, p)
        if rn <= tol * nb:
            return SolveResult(x=x, iters=k + 1, converged=True, rel_res=hist[-1], history=hist)
        z = r if M is None else np.asarray(M(r), dtype=dtype)
        rho_new = r @ z
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return SolveResult(x=x, iters=max_iter, converged=False, rel_res=hist[-1],
                       history=hist, status="max_iter")


def jacobi(A):
    """The Jacobi preconditioner ``z = r / diag(A)``."""
    dinv = 1.0 / A.diagonal()
    return lambda r: dinv.astype(r.dtype) * r


def fcg(A, b, M, x0=None, tol=1e-6, max_iter=10000, dtype=np.float64, callback=None):
    """Flexible CG with the Golub-Ye beta; ``M(r)`` may change from call to call."""
    b = np.asarray(b, dtype=dtype)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=dtype).copy()
    r = b - A @ x if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    if nb == 0:
        return SolveResult(x=x, iters=0, converged=True, rel_res=0.0, history=[0.0])
    z = np.asarray(M(r), dtype=dtype)
    zr = z @ r
    p = z.copy()
    hist = [float(np.linalg.norm(r) / nb)]
    if hist[0] <= tol:
        return SolveResult(x=x, iters=0, converged=True, rel_res=hist[0], history=hist)
    for k in range(max_iter):
        q = A @ p
        pq = p @ q
        if not (pq > 0) or not np.isfinite(pq):
            return SolveResult(x=x, iters=k, converged=False, rel_res=hist[-1],
                               history=hist, status="breakdown")
        alpha = zr / pq
        x += alpha * p
        r_old = r
        r = r - alpha * q
        rn = np.linalg.norm(r)
        hist.append(float(rn / nb))
        if callback is not None:
            callback(k, x, r, p)
        if rn <= tol * nb:
            return SolveResult(x=x, iters=k + 1, converged=True, rel_res=hist[-1], history=hist)
        z_new = np.asarray(M(r), dtype=dtype)
        beta = (z_new @ (r - r_old)) / zr
        zr = z_new @ r
        p = z_new + beta * p
    return SolveResult(x=x, iters=max_iter, converged=False, rel_res=hist[-1],
                       history=hist, status="max_iter")


def iterative_refinement(A, b, tol=1e-8, inner_tol=1e-4, max_outer=10,
                         inner_max_iter=100000, x0=None):
    """Mixed-precision refinement: FP64 residuals, FP32 CG corrections.

    Each outer step forms ``r = b - A x`` in FP64 and stops once
    ``||r|| <= tol*||b||``; otherwise it solves ``A d = r/||r||`` with FP32 CG to
    ``inner_tol`` and adds ``||r|| d`` to the FP64 iterate.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    A32 = A.astype(np.float32)
    nb = np.linalg.norm(b)
    hist = []
    total = 0
    for outer in range(max_outer + 1):
        r = b - A @ x
        rn = np.linalg.norm(r)
        hist.append(float(rn / nb))
        if rn <= tol * nb:
            return SolveResult(x=x, iters=total, converged=True, rel_res=hist[-1],
                               history=hist, outer=outer)
        if outer == max_outer:
            break
        res = cg(A32, (r / rn).astype(np.float32), tol=inner_tol,
                 max_iter=inner_max_iter, dtype=np.float32)
        total += res.iters
        x += rn * res.x.astype(np.float64)
    return SolveResult(x=x, iters=total, converged=False, rel_res=hist[-1],
                       history=hist, status="max_iter", outer=max_outer)
