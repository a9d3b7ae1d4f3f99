"""Preconditioned conjugate gradients (oracle).

Test infrastructure only.  The paper applies the full multigrid cycle once
per iteration of the Conjugate Gradient method (Section 6).  It gives no
further details, so this is the textbook Hestenes-Stiefel recurrence:
x_0 = 0, r_0 = b, z = M^{-1} r, p = z; per iteration q = A p,
alpha = (r.z)/(p.q), x += alpha p, r -= alpha q, stop when
||r||_2 <= tol ||b||_2, z = M^{-1} r, beta = (r.z)_new/(r.z)_old,
p = z + beta p.  The iteration count is the number of products with A.
"""
from __future__ import annotations

import numpy as np


class Breakdown(RuntimeError):
    pass


def pcg(apply_A, apply_M, b, tol, max_iter=1000):
    """Returns (x, iterations, relative residual history, converged)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.sqrt(b @ b))
    if bnorm == 0.0:
        return x, 0, [0.0], True
    r = b.copy()
    z = apply_M(r)
    p = z.copy()
    rho = float(r @ z)
    hist = [1.0]
    for k in range(1, max_iter + 1):
        q = apply_A(p)
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            raise Breakdown(f"p.Ap = {pq} at iteration {k}")
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        rel = float(np.sqrt(r @ r)) / bnorm
        hist.append(rel)
        if rel <= tol:
            return x, k, hist, True
        z = apply_M(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, max_iter, hist, False


def two_sum(a, b):
    """Error-free sum (Knuth): s = fl(a + b) and e with s + e = a + b exactly."""
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def pcg_restarted(apply_A, apply_M, b, tol, max_iter=1000, max_restarts=5, residual=None):
    """PCG whose stopping test is confirmed on the true residual b - A x.

    When the recurrence residual reaches tol but the true one does not, PCG
    restarts with the true residual as right-hand side and solves for a
    correction from zero (at most max_restarts times, and only while each
    restart at least halves the true residual).

    The solution is held as the unevaluated sum hi + lo of two doubles: each
    correction is added with an error-free sum, its rounding error kept in
    lo.  residual(hi, lo) returns b - A (hi + lo); the default evaluates A hi
    and A lo in FP64.  Section 6 observes an accuracy floor that grows with
    the condition number and ascribes it to FP64 round-off; with an
    extended-precision residual (fem.residual_extended) the refinement
    removes it and the solution becomes accurate to FP64 rounding, while a
    plain FP64 residual leaves the floor where rounding the iterate puts it.
    Returns (fl(hi + lo), iterations, relative residual of hi + lo,
    converged, restarts); converged = False at the floor, at max_iter or
    after max_restarts."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.sqrt(b @ b))
    hi = np.zeros_like(b)
    lo = np.zeros_like(b)
    if bnorm == 0.0:
        return hi, 0, 0.0, True, 0
    if residual is None:
        def residual(h, l):
            return (b - apply_A(h)) - apply_A(l)
    total = 0
    prev = np.inf
    restarts = 0
    while True:
        r = residual(hi, lo)
        rel = float(np.sqrt(r @ r)) / bnorm
        if rel <= tol:
            return hi + lo, total, rel, True, restarts
        if total >= max_iter or restarts > max_restarts or rel > 0.5 * prev:
            return hi + lo, total, rel, False, restarts
        if total > 0:
            restarts += 1
        prev = rel
        dx, it, _, _ = pcg(apply_A, apply_M, r, tol * bnorm / (rel * bnorm), max_iter - total)
        hi, e = two_sum(hi, dx)
        lo = lo + e
        total += it
