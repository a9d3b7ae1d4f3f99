"""Vertical extrapolation operator E~ (paper Section 5.4, Fig. vertical_interpolation).

Test infrastructure (oracle).

E~ = [I; F]: a top node keeps its own value; every other node is projected
straight up onto the top-surface triangle mesh and takes the linear
interpolant of the three surface values of the triangle it lands in, so each
row has at most three entries.  The paper's "R^{m'} -> R^{m_bar}" is read as
the map from the m' free surface values to all n free node values.

Readings (the paper is silent on them):
* surface triangles are the tetrahedron faces whose three vertices are top
  nodes, numbered in ascending order of their sorted vertex triple;
* barycentric coordinates of the point p in triangle (p1, p2, p3):
    det = (y2-y3)(x1-x3) + (x3-x2)(y1-y3)
    l1  = ((y2-y3)(x-x3) + (x3-x2)(y-y3)) / det
    l2  = ((y3-y1)(x-x3) + (x1-x3)(y-y3)) / det
    l3  = (1 - l1) - l2;
* p lies in a triangle when every l >= -1e-12; among several such triangles
  the one with the smallest number wins; a node in none is an error;
* weights with |l| <= 1e-12 become zero and the rest are divided by their
  sum (l1 + l2) + l3;
* a Dirichlet surface node (the pinned node x_0) has no column: its weight is
  dropped without renormalisation, which is E~ restricted to the space with
  phi(x_0) = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

TOL_INSIDE = 1e-12


def top_triangles(tets, top):
    """Surface triangles: tetrahedron faces with all three vertices on top."""
    faces = np.concatenate([tets[:, [0, 1, 2]], tets[:, [0, 1, 3]],
                            tets[:, [0, 2, 3]], tets[:, [1, 2, 3]]])
    faces = faces[top[faces].all(axis=1)]
    faces = np.sort(faces, axis=1)
    return np.unique(faces, axis=0)


def barycentric(xy, tri_xy):
    """Barycentric coordinates of points xy [k,2] in triangles tri_xy [k,3,2]."""
    x, y = xy[:, 0], xy[:, 1]
    x1, y1 = tri_xy[:, 0, 0], tri_xy[:, 0, 1]
    x2, y2 = tri_xy[:, 1, 0], tri_xy[:, 1, 1]
    x3, y3 = tri_xy[:, 2, 0], tri_xy[:, 2, 1]
    det = (y2 - y3) * (x1 - x3) + (x3 - x2) * (y1 - y3)
    l1 = ((y2 - y3) * (x - x3) + (x3 - x2) * (y - y3)) / det
    l2 = ((y3 - y1) * (x - x3) + (x1 - x3) * (y - y3)) / det
    l3 = (1.0 - l1) - l2
    return np.stack([l1, l2, l3], axis=1)


def locate(points_xy, tri, xyz, ngrid=None):
    """Smallest-numbered triangle containing each point (or -1), and the
    barycentric coordinates there.  A bucket grid only narrows the candidate
    list; the answer equals a brute-force scan over all triangles."""
    txy = xyz[tri][:, :, :2]
    lo = txy.min(axis=1)
    hi = txy.max(axis=1)
    gmin = np.minimum(lo.min(axis=0), points_xy.min(axis=0))
    gmax = np.maximum(hi.max(axis=0), points_xy.max(axis=0))
    if ngrid is None:
        ngrid = max(1, int(np.sqrt(tri.shape[0] / 2.0)))
    span = np.maximum(gmax - gmin, 1e-300)
    pad = 1e-9 * span

    def cell(v):
        c = np.floor((v - gmin) / span * ngrid).astype(np.int64)
        return np.clip(c, 0, ngrid - 1)

    c_lo = cell(lo - pad)
    c_hi = cell(hi + pad)
    # triangle -> cells (bounding boxes cover only a few cells)
    reg_tri, reg_cell = [], []
    for dx in range(int((c_hi[:, 0] - c_lo[:, 0]).max()) + 1):
        for dy in range(int((c_hi[:, 1] - c_lo[:, 1]).max()) + 1):
            cx = c_lo[:, 0] + dx
            cy = c_lo[:, 1] + dy
            ok = (cx <= c_hi[:, 0]) & (cy <= c_hi[:, 1])
            reg_tri.append(np.nonzero(ok)[0])
            reg_cell.append(cy[ok] * ngrid + cx[ok])
    reg_tri = np.concatenate(reg_tri)
    reg_cell = np.concatenate(reg_cell)
    o = np.lexsort((reg_tri, reg_cell))
    reg_tri, reg_cell = reg_tri[o], reg_cell[o]
    cstart = np.searchsorted(reg_cell, np.arange(ngrid * ngrid + 1))

    pc = cell(points_xy)
    pcell = pc[:, 1] * ngrid + pc[:, 0]
    cnt = cstart[pcell + 1] - cstart[pcell]
    npts = points_xy.shape[0]
    best = np.full(npts, -1, dtype=np.int64)
    lam = np.zeros((npts, 3))
    for k in range(int(cnt.max()) if npts else 0):
        live = np.nonzero(cnt > k)[0]
        t = reg_tri[cstart[pcell[live]] + k]
        l = barycentric(points_xy[live], txy[t])
        inside = (l >= -TOL_INSIDE).all(axis=1)
        take = inside & ((best[live] < 0) | (t < best[live]))
        best[live[take]] = t[take]
        lam[live[take]] = l[take]
    return best, lam


def vertical_extrapolation(xyz, tets, top, node_order, dirichlet):
    """E~ as a CSR matrix with rows in ``node_order`` (the free nodes in
    device order) and columns numbered by the position of each free top node
    in ``node_order`` (the top block comes first in that order).

    Returns (E CSR [n_free, m'], triangle index per row (-1 for top rows)).
    """
    n_free = node_order.size
    pos = np.full(xyz.shape[0], -1, dtype=np.int64)
    pos[node_order] = np.arange(n_free)
    surf = top & ~dirichlet
    m = int(np.count_nonzero(surf[node_order]))
    tri = top_triangles(tets, top)
    rows, cols, vals = [], [], []
    is_top = top[node_order]
    # top rows: identity
    r_top = np.nonzero(is_top)[0]
    rows.append(r_top)
    cols.append(pos[node_order[r_top]])
    vals.append(np.ones(r_top.size))
    # other rows: project up and interpolate
    r_in = np.nonzero(~is_top)[0]
    nodes = node_order[r_in]
    which, lam = locate(xyz[nodes, :2], tri, xyz)
    if np.any(which < 0):
        bad = int(nodes[np.nonzero(which < 0)[0][0]])
        raise ValueError(f"node {bad} does not project onto the top surface")
    lam = np.where(np.abs(lam) <= TOL_INSIDE, 0.0, lam)
    s = (lam[:, 0] + lam[:, 1]) + lam[:, 2]
    lam = lam / s[:, None]
    verts = tri[which]
    for k in range(3):
        v = verts[:, k]
        keep = (lam[:, k] != 0.0) & ~dirichlet[v]
        rows.append(r_in[keep])
        cols.append(pos[v[keep]])
        vals.append(lam[keep, k])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    E = sp.csr_matrix((vals, (rows, cols)), shape=(n_free, m))
    E.sort_indices()
    tri_of_row = np.full(n_free, -1, dtype=np.int64)
    tri_of_row[r_in] = which
    return E, tri_of_row


def sspai_refit(E0, A, n_top):
    """The sparse-approximate-inverse alternative to the projection (Section
    5.4, second approach): E~ = [I; F] keeps the pattern of the projected
    E~, and the entries of F are refitted from the operator.

    The exact extrapolation is E = [I; -A_bar^{-1} C^T] (Section 5.3), with
    A_bar the non-top block of A_UU and C^T its coupling block (non-top rows,
    top columns).  Column i of F is fitted on its own: with J the non-top
    rows where column i of the pattern is non-empty, v = F[J, i] solves the
    restriction of A_bar f_i = -C^T e_i to J,
        A_bar[J, J] v = -C^T[J, i],
    entries outside J staying zero.  Reading: the text writes the fitting
    objective as |F^T A_bar - C| while its decoupled column systems carry
    -r_i on the right; the exact E above fixes the sign, and the column
    systems are what is solved here.  Each dense system is solved by
    Cholesky (A_bar[J, J] is a principal submatrix of a symmetric positive
    definite matrix).

    E0: n x m' CSR in storage order (top rows first, identity there); A: the
    standard-form A_UU in the same order.  Returns a new CSR with the same
    pattern."""
    import scipy.linalg

    E = E0.tocsr().copy()
    E.sort_indices()
    A = A.tocsr()
    Ec = E.tocsc()
    Ec.sort_indices()
    for i in range(E.shape[1]):
        rows = Ec.indices[Ec.indptr[i]:Ec.indptr[i + 1]]
        J = rows[rows >= n_top]
        if J.size == 0:
            continue
        G = A[J][:, J].toarray()
        rhs = -A[J, i].toarray().ravel()
        v = scipy.linalg.cho_solve(scipy.linalg.cho_factor(G, lower=True), rhs)
        for r, val in zip(J, v):
            k = E.indptr[r] + np.searchsorted(E.indices[E.indptr[r]:E.indptr[r + 1]], i)
            E.data[k] = val
    return E
