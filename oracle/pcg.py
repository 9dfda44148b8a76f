"""Preconditioned conjugate gradients (oracle, float64).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Standard PCG (Saad 2003, Alg. 9.1; the paper's Sec. 3 convergence bound and
Sec. 5 solve loop) with this build's run-time policy:

  setup:  x = x0 (default 0), r = b - A x, z = M r, p = z, rho = r.z
  each iteration k = 1, 2, ...:
      q = A p;  alpha = rho / (p.q);  x += alpha p;  r -= alpha q
      if k % recompute_every == 0 or forced:  r = b - A x   (residual replacement)
      stop (CONVERGED) when ||r|| <= tol * ||b|| on a replaced (true) residual;
          a recurrence residual that passes forces replacement next iteration
      stop (STAGNATED) when k % 100 == 0 and ||r_k|| > 0.5 ||r_{k-100}||
      stop (MAXITER) when k == max_iter
      z = M r;  rho' = r.z;  stop (NOT_SPD) unless rho' > 0 and finite
      beta = rho' / rho;  p = z + beta p
  iterations = number of SpMVs in the loop.

The stagnation window and the Jacobi fallback (on any of NOT_SPD, STAGNATED,
MAXITER) are this build's additions: the paper enforces no SPD property on M
and has no fallback.

fp32_iteration=True follows the paper's precision split (Sec. 6.3;
Supplementary "Precision"): the iteration's operator and vectors are float32
and only its scalars float64.  q = A p uses A with every entry rounded to
float32; r, z, p and q are held in float32 (each computed in float64 from
float32 operands and rounded once); x, every inner product, norm and step
size stay float64, and the replaced (true) residual b - A x uses the float64
operator.  At tight tolerances the split costs iterations, mostly through
the rounded operator: the recurrence follows A rounded to float32 while the
stop is judged on the float64 A.  The default is float64 throughout.
"""
from __future__ import annotations

import math
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

CONVERGED, NOT_SPD, STAGNATED, MAXITER, FELL_BACK = 1, 2, 4, 8, 16


def pcg(A, b: np.ndarray, M: Optional[Callable] = None, tol: float = 1e-6,
        max_iter: int = 10000, recompute_every: int = 25, x0: Optional[np.ndarray] = None,
        stagnation: bool = True, bnorm: Optional[float] = None, fp32_iteration: bool = False):
    """Returns (x, iterations, flags, relres history)."""
    b = np.asarray(b, dtype=np.float64)
    v = (lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)) if fp32_iteration \
        else (lambda a: a)
    Aq = A
    if fp32_iteration:
        if sp.issparse(A):
            Aq = A.copy()
            Aq.data = Aq.data.astype(np.float32).astype(np.float64)
        else:
            Aq = np.asarray(A, np.float64).astype(np.float32).astype(np.float64)
    M0 = (lambda r: r.copy()) if M is None else M
    Mf = lambda r: v(M0(r))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = v(b - A @ x)
    if bnorm is None:
        bnorm = float(np.sqrt(b @ b))
    target = tol * bnorm
    hist = [float(np.sqrt(r @ r)) / bnorm if bnorm > 0 else 0.0]
    if math.sqrt(r @ r) <= target:
        return x, 0, CONVERGED, hist
    z = Mf(r)
    rho = float(r @ z)
    if not (rho > 0 and math.isfinite(rho)):
        return x, 0, NOT_SPD, hist
    p = z.copy()
    k, flags = 0, 0
    force = False
    last_window = math.sqrt(r @ r)       # ||r_0||: the first window's reference
    while True:
        if k >= max_iter:
            flags = MAXITER
            break
        q = v(Aq @ p)
        alpha = rho / float(p @ q)
        x = x + alpha * p
        r = v(r - alpha * q)
        k += 1
        replaced = force or bool(recompute_every and k % recompute_every == 0)
        if replaced:
            r = v(b - A @ x)
        force = False
        rn = math.sqrt(float(r @ r))
        hist.append(rn / bnorm)
        if rn <= target:
            if replaced:
                flags = CONVERGED
                break
            force = True   # confirm on the true residual next iteration
        if stagnation and k % 100 == 0:
            if rn > 0.5 * last_window:
                flags = STAGNATED
                break
            last_window = rn
        if k >= max_iter:
            flags = MAXITER
            break
        z = Mf(r)
        rho_new = float(r @ z)
        if not (rho_new > 0 and math.isfinite(rho_new)):
            flags = NOT_SPD
            break
        beta = rho_new / rho
        rho = rho_new
        p = v(z + beta * p)
    return x, k, flags, hist


def jacobi(A) -> Callable:
    """M = diag(A)^-1 (Jacobi preconditioner, the paper's GPU baseline)."""
    d = np.asarray(A.diagonal(), dtype=np.float64)
    return lambda r: r / d


def solve_with_fallback(A, b, M: Callable, tol: float = 1e-6, max_iter: int = 10000,
                        recompute_every: int = 25, stagnation: bool = True, fp32_iteration: bool = False):
    """Learned-M PCG; a frame that did not converge (NOT_SPD, STAGNATED or
    MAXITER: positivity lost, less than a 2x drop of ||r|| over 100
    iterations, or the iteration cap) restarts as Jacobi-PCG warm-started from
    the current x, to the same target tol * ||b||, with the same cap and no
    stagnation check.  Iterations add up; the flags of both passes are kept."""
    x, k, flags, hist = pcg(A, b, M, tol, max_iter, recompute_every, stagnation=stagnation,
                            fp32_iteration=fp32_iteration)
    if not flags & CONVERGED:
        bn = float(np.sqrt(b @ b))
        x, k2, f2, h2 = pcg(A, b, jacobi(A), tol, max_iter, recompute_every, x0=x,
                            stagnation=False, bnorm=bn, fp32_iteration=fp32_iteration)
        return x, k + k2, f2 | FELL_BACK | flags, hist + h2[1:]
    return x, k, flags, hist
