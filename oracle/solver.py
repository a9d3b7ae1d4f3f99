"""End-to-end oracle: setup in the device node order, and solve.

Test infrastructure only.

Order of the free unknowns ("storage order"): top block first (paper
eq. phi_decomposition), each block in locality order, then stably sorted by
the colour of A_UU (greedy in smallest-last order, see ordering.py).  The
non-top block is the matrix A_bar of eq. equation_decomposition; its colouring
is the restriction of the colouring of A_UU.  The surface operator
S = E~^T A E~ (indexed in the top block's storage order) is stored in the
block multicolour (patch) order of the coarse levels, its spatial order being
the locality order of the top nodes; E~'s columns follow that order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import amg, extrap, fem, ordering, pcg, precond


@dataclass
class OracleSetup:
    mode: str
    n_nodes: int
    pin: int
    perm: np.ndarray          # storage position -> natural node index
    n_top: int                # free top unknowns (= m')
    Aoff: sp.csr_matrix       # off-diagonals of A_UU, storage order
    d: np.ndarray             # deficit, storage order
    A: sp.csr_matrix          # standard form A_UU, storage order
    diag: np.ndarray
    colour: np.ndarray        # colour of every storage row (sorted within each block)
    rank: np.ndarray          # position of every storage row in the locality order
    E: sp.csr_matrix | None   # n x m', columns in S storage order
    S_perm: np.ndarray | None  # S storage position -> top-block position
    S_levels: list | None
    Abar_levels: list
    mass: sp.csr_matrix       # full consistent mass matrix, natural order
    xyz: np.ndarray
    top: np.ndarray
    coarse_max: int = 8192    # hierarchy parameters (also for the SA baseline)
    max_levels: int = 10
    extrapolation: str = "projection"

    @property
    def n(self):
        return self.perm.size


def setup(mesh, mode="N", coarse_max=8192, max_levels=10, alpha=0.0, extrapolation="projection"):
    """Assembly (Section 3), E~ (Section 5.4) and both SA hierarchies (Section 6).
    mode 'N' (point condition), 'D' (Dirichlet top) or 'R' (Robin top with
    coefficient alpha > 0, the free-surface condition of Section 2).
    extrapolation: 'projection' (the vertical projection of Section 5.4) or
    'sspai' (its pattern with F refitted from A, the second approach of
    Section 5.4)."""
    if extrapolation not in ("projection", "sspai"):
        raise ValueError(extrapolation)
    xyz, tets, top = mesh.xyz, mesh.tets, mesh.top
    n_nodes = xyz.shape[0]
    _, Aoff_full = fem.assemble_stiffness(xyz, tets)
    d_robin = np.zeros(n_nodes)
    if mode == "R":
        if not alpha > 0.0:
            raise ValueError("the Robin coefficient must be positive")
        Moff, L = fem.top_surface_mass(xyz, extrap.top_triangles(tets, top))
        Aoff_full, d_robin = fem.add_robin(Aoff_full, Moff, L, alpha)
    pin = fem.pin_node(xyz, top) if mode == "N" else -1
    D = fem.dirichlet_set(xyz, top, mode, pin)
    free = ~D
    # locality order and colouring of A_UU (indices in natural numbering)
    loc = ordering.locality_order(xyz, top, free)
    U, Auu_nat, d_nat = fem.reduce_to_unknowns(Aoff_full, D)
    d_nat = d_nat + d_robin[U]
    pos_in_U = np.full(n_nodes, -1, dtype=np.int64)
    pos_in_U[U] = np.arange(U.size)
    loc_u = pos_in_U[loc]
    colour_u = ordering.colouring(Auu_nat)
    block = np.where(top[U], 0, 1)
    order_u = ordering.colour_sorted(loc_u, colour_u, block)
    perm = U[order_u]
    Aoff = ordering_permute(Auu_nat, order_u)
    d = d_nat[order_u] + 0.0
    A = fem.full_matrix(Aoff, d)
    diag = fem.diagonal_of(Aoff, d)
    colour = colour_u[order_u]
    n_top = int(np.count_nonzero(top[perm]))
    n = perm.size
    loc_pos = np.full(n_nodes, -1, dtype=np.int64)
    loc_pos[loc] = np.arange(loc.size)
    rank = loc_pos[perm]      # the top block ranks first (block 0 of the locality key)

    # surface branch: E~, S = E~^T A E~ and its hierarchy (mode N only)
    E = None
    S_perm = None
    S_levels = None
    if n_top > 0:
        E0, _ = extrap.vertical_extrapolation(xyz, tets, top, perm, D)
        if extrapolation == "sspai":
            E0 = extrap.sspai_refit(E0, A, n_top)
        S0 = amg.structural_product(E0.T.tocsr(), A, E0)
        S_perm, S_arr = amg.patch_level(S0, rank[:n_top])
        E = E0[:, S_perm].tocsr()
        E.sort_indices()
        # near-kernel of the vertically lumped operator: the constant and the
        # two horizontal coordinates (P1 extrapolation of a linear function
        # of x, y has no vertical gradient, so it lies in ker A_0, Section 4)
        top_nodes = perm[:n_top][S_perm]
        B0 = np.column_stack([np.ones(n_top), xyz[top_nodes, 0], xyz[top_nodes, 1]])
        S_levels = amg.build_hierarchy(amg.permute(S0, S_perm), S_arr["colour"], B0, coarse_max, max_levels,
                                       rank0=S_arr["rank"],
                                       first={k: S_arr[k] for k in ("patch", "pcolour", "lcolour")})

    # interior branch: A_bar = non-top block
    Abar = A[n_top:, n_top:].tocsr()
    Abar.sort_indices()
    Abar_levels = amg.build_hierarchy(Abar, colour[n_top:], None, coarse_max, max_levels,
                                      rank0=rank[n_top:] - n_top)

    return OracleSetup(mode=mode, n_nodes=n_nodes, pin=pin, perm=perm, n_top=n_top,
                       Aoff=Aoff, d=d, A=A, diag=diag, colour=colour, rank=rank, E=E, S_perm=S_perm,
                       S_levels=S_levels, Abar_levels=Abar_levels,
                       mass=fem.assemble_mass(xyz, tets), xyz=xyz, top=top, coarse_max=coarse_max,
                       max_levels=max_levels, extrapolation=extrapolation)


def ordering_permute(A, order):
    B = A.tocsr()[order][:, order].tocsr()
    B.sort_indices()
    return B


def apply_A(s: OracleSetup, x):
    """A_UU x in difference form (the operator CG solves)."""
    return fem.apply_difference_form(s.Aoff, s.d, x)


def rhs_from_field(s: OracleSetup, f_nodal):
    """b = M f (eq. Ax=b) restricted to the free nodes, storage order.  In
    mode N the Neumann problem needs int f = 0; b is first made orthogonal to
    constants by subtracting (sum b / sum w) w, w = M 1 (reading)."""
    b = s.mass @ f_nodal
    if s.mode == "N":
        w = s.mass @ np.ones(s.n_nodes)
        b = b - (b.sum() / w.sum()) * w
    return b[s.perm]


def rhs_from_solution(s: OracleSetup, x_nodal):
    """b = A_UU x* for a chosen solution x* (the paper's error protocol,
    Section 6: choose a solution and multiply by the matrix).  Values of x*
    at Dirichlet nodes are ignored (taken as zero)."""
    return apply_A(s, x_nodal[s.perm])


def to_natural(s: OracleSetup, x):
    out = np.zeros(s.n_nodes)
    out[s.perm] = x
    return out


def solve(s: OracleSetup, b, tol=1e-8, pc="vl_as", max_iter=1000):
    """PCG on A_UU x = b (storage order), stopping test confirmed on the true
    residual of the extended iterate, evaluated in extended precision.
    Returns (x, iterations, that relative residual, converged)."""
    M = precond.make(s, pc)
    x, it, rel, ok, _ = pcg.pcg_restarted(lambda v: apply_A(s, v), M, b, tol, max_iter,
                                          residual=lambda hi, lo: fem.residual_extended(s.Aoff, s.d, b, hi, lo))
    return x, it, rel, ok
