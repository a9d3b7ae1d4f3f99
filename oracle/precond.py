"""Preconditioners of Section 6 (oracle).

Test infrastructure only.

* 'vl_sor' -- vertical lumping as the first coarsening of an ordinary
              multigrid cycle with one forward SOR sweep on A before and one
              backward sweep after (Section 6, second preconditioner):
              x = GS_fwd(A, r); x += E~ Vcyc_S(E~^T (r - A x)); x = GS_bwd(A, r, x).
* 'vl_as'  -- that cycle with the additive smoother included (Section 6,
              third preconditioner; Section 5.5 for the smoother):
              z = vl_sor(r) + Z Vcyc_Abar(Z^T r), Z = [0; I].
              Reading: Section 6 describes the third preconditioner as the
              vertical-lumping cycle combined with the smoother and compares
              the preconditioner with and without it; taking the sum keeps
              the SOR cycle of the second preconditioner and adds the second
              term of eq. ourpreconditioner with A_bar^{-1} replaced by one
              V-cycle.  The sum of two symmetric positive definite operators
              is one, so CG applies.
* 'vl_add' -- eq. ourpreconditioner on its own, no SOR:
              z = E~ Vcyc_S(E~^T r) + Z Vcyc_Abar(Z^T r).
              The two terms are independent; with exact solves in both and
              the exact extrapolation E this is A^{-1} (eq. E multigrid).
* 'sa'     -- one smoothed aggregation V-cycle on the whole A (the first
              preconditioner of Section 6, the paper's baseline, which shows
              eps-dependent plateaus).
* 'jacobi' -- z = r / diag(A).
* 'none'   -- z = r.
In mode D the surface branch is empty (all top values are fixed): 'vl_sor'
is then one symmetric Gauss-Seidel sweep and 'vl_add' the additive smoother
alone.
"""
from __future__ import annotations

import numpy as np

from . import amg


def _additive_smoother(s, r):
    """Z Vcyc_Abar(Z^T r): one V-cycle on the non-top block, zero on top."""
    z = np.zeros_like(r)
    z[s.n_top:] = amg.vcycle(s.Abar_levels, r[s.n_top:])
    return z


def _vl_add(s):
    def apply(r):
        z = _additive_smoother(s, r)
        if s.n_top > 0:
            z += s.E @ amg.vcycle(s.S_levels, s.E.T @ r)
        return z
    return apply


def _vl_as(s):
    sor = _vl_sor(s)

    def apply(r):
        return sor(r) + _additive_smoother(s, r)
    return apply


def _vl_sor(s):
    def apply(r):
        x = amg.gs_sweep(s.A, s.diag, s.colour, r, np.zeros_like(r), forward=True)
        if s.n_top > 0:
            res = r - s.A @ x
            x = x + s.E @ amg.vcycle(s.S_levels, s.E.T @ res)
        x = amg.gs_sweep(s.A, s.diag, s.colour, r, x, forward=False)
        return x
    return apply


def sa_levels(s, coarse_max=None, max_levels=None):
    """The smoothed aggregation hierarchy of the whole A_UU, built in the
    storage order (top block first, each block colour-sorted; the fine-level
    sweeps take colour c of both blocks at once).  Reading: the paper fixes no
    node order for its baseline; this is the order of the lumping method."""
    if getattr(s, "_sa_levels", None) is None:
        s._sa_levels = amg.build_hierarchy(s.A, s.colour, None, coarse_max or s.coarse_max,
                                           max_levels or s.max_levels, rank0=s.rank)
    return s._sa_levels


def _sa(s):
    levels = sa_levels(s)

    def apply(r):
        return amg.vcycle(levels, r)
    return apply


def make(s, pc):
    if pc == "sa":
        return _sa(s)
    if pc == "vl_as":
        return _vl_as(s)
    if pc == "vl_add":
        return _vl_add(s)
    if pc == "vl_sor":
        return _vl_sor(s)
    if pc == "jacobi":
        return lambda r: r / s.diag
    if pc == "none":
        return lambda r: r.copy()
    raise ValueError(pc)
