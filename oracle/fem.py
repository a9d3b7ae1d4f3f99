"""P1 finite-element assembly (paper Section 3).

Test infrastructure (oracle): plain FP64 NumPy/SciPy, no GPU code.

The stiffness matrix is assembled in physical coordinates.  With x = L x',
z = H z' this equals (L^2/H) (A_0 + eps^2 A_H), the rescaled operator of
eq. (rescaled Poisson), so relative residuals and iterates are unchanged
(Section 4 splits A_eps = A_0 + eps^2 A_H).

Arithmetic order is fixed so that the result is reproducible bit for bit:
every edge value is a sequential sum over its elements in ascending element
index, and every row sum runs over ascending column index.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# local edge pairs (a, b), a < b, of a tetrahedron
_PAIRS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _cross(a, b):
    return np.stack([a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1],
                     a[:, 2] * b[:, 0] - a[:, 0] * b[:, 2],
                     a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]], axis=1)


def _dot(a, b):
    return a[:, 0] * b[:, 0] + a[:, 1] * b[:, 1] + a[:, 2] * b[:, 2]


def element_geometry(xyz, tets):
    """Scaled barycentric gradients of every tetrahedron.

    With e_k = X_k - X_0, the gradients of the P1 basis functions N_1..N_3
    are c_1/det, c_2/det, c_3/det with c_1 = e_2 x e_3, c_2 = e_3 x e_1,
    c_3 = e_1 x e_2 and det = e_1 . c_1 = 6 vol; grad N_0 = -(sum of the
    others).  Returns (c [T,4,3], det [T]).
    """
    x0 = xyz[tets[:, 0]]
    e1 = xyz[tets[:, 1]] - x0
    e2 = xyz[tets[:, 2]] - x0
    e3 = xyz[tets[:, 3]] - x0
    c1 = _cross(e2, e3)
    c2 = _cross(e3, e1)
    c3 = _cross(e1, e2)
    c0 = -((c1 + c2) + c3)
    det = _dot(e1, c1)
    return np.stack([c0, c1, c2, c3], axis=1), det


def element_stiffness(xyz, tets, weights=(1.0, 1.0, 1.0)):
    """K_e[a, b] = int_e grad N_a . W grad N_b = (c_a . W c_b) / (6 det).

    ``weights`` multiplies the x, y, z derivative products (1, 1, 1 gives
    the Laplacian of eq. Ax=b; (0, 0, 1) and (1, 1, 0) give the vertical and
    horizontal parts A_0 and A_H of Section 4).  Returns [T, 4, 4].
    """
    c, det = element_geometry(xyz, tets)
    if np.any(det <= 0.0):
        bad = int(np.nonzero(det <= 0.0)[0][0])
        raise ValueError(f"tetrahedron {bad} is not positively oriented")
    wx, wy, wz = weights
    K = np.empty((tets.shape[0], 4, 4))
    for a in range(4):
        for b in range(4):
            ca, cb = c[:, a], c[:, b]
            dot = (wx * (ca[:, 0] * cb[:, 0]) + wy * (ca[:, 1] * cb[:, 1])) + wz * (ca[:, 2] * cb[:, 2])
            K[:, a, b] = dot / (6.0 * det)
    return K


def element_mass(xyz, tets):
    """Consistent P1 mass matrix: M_e[a, b] = vol/20 (1 + delta_ab)."""
    _, det = element_geometry(xyz, tets)
    vol = det / 6.0
    M = np.repeat((vol / 20.0)[:, None, None], 4, axis=1).repeat(4, axis=2)
    M = M * (np.ones((4, 4)) + np.eye(4))[None]
    return M


def _sequential_sum_by_key(keys, values, nkeys):
    """out[k] = values[i1] + values[i2] + ... over the entries with key k, in
    the order they appear (a strict left-to-right sum, vectorised across keys)."""
    order = np.argsort(keys, kind="stable")
    k_sorted = keys[order]
    v_sorted = values[order]
    start = np.searchsorted(k_sorted, np.arange(nkeys), side="left")
    count = np.bincount(k_sorted, minlength=nkeys)
    out = np.zeros(nkeys)
    for step in range(int(count.max()) if count.size else 0):
        live = np.nonzero(count > step)[0]
        out[live] = out[live] + v_sorted[start[live] + step]
    return out


def edge_list(n, tets):
    """Unique mesh edges (i < j), sorted by (i, j)."""
    e = np.concatenate([np.stack([tets[:, a], tets[:, b]], axis=1) for a, b in _PAIRS])
    e = np.sort(e, axis=1)
    key = np.unique(e[:, 0] * n + e[:, 1])
    return np.stack([key // n, key % n], axis=1)


def assemble_offdiag(n, tets, Ke):
    """Off-diagonal part of sum_e K_e on the mesh edge graph (numerical zeros
    kept).  Each edge value is a left-to-right sum over the elements that
    contain it, in ascending element index.  Returns a symmetric CSR matrix
    with an empty diagonal and sorted column indices."""
    edges = edge_list(n, tets)
    ekey = edges[:, 0] * n + edges[:, 1]
    T = tets.shape[0]
    # contributions grouped by element (ascending), then by local pair
    vals = np.empty((T, 6))
    keys = np.empty((T, 6), dtype=np.int64)
    for p, (a, b) in enumerate(_PAIRS):
        i = np.minimum(tets[:, a], tets[:, b])
        j = np.maximum(tets[:, a], tets[:, b])
        keys[:, p] = np.searchsorted(ekey, i * n + j)
        vals[:, p] = Ke[:, a, b]
    w = _sequential_sum_by_key(keys.ravel(), vals.ravel(), edges.shape[0])
    rows = np.concatenate([edges[:, 0], edges[:, 1]])
    cols = np.concatenate([edges[:, 1], edges[:, 0]])
    data = np.concatenate([w, w])
    A = sp.csr_matrix((data, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A


def row_sums(Aoff):
    """Left-to-right row sums of a CSR matrix in ascending column order."""
    n = Aoff.shape[0]
    rows = np.repeat(np.arange(n), np.diff(Aoff.indptr))
    return _sequential_sum_by_key(rows, Aoff.data, n)


def assemble_stiffness(xyz, tets, weights=(1.0, 1.0, 1.0)):
    """Full stiffness matrix A of eq. Ax=b (Neumann everywhere).

    The diagonal is a_ii = -sum_{j != i} a_ij: the P1 basis is a partition of
    unity, so its gradients sum to zero and every row of A sums to zero.
    Returns (A_full CSR, Aoff CSR without diagonal)."""
    n = xyz.shape[0]
    Ke = element_stiffness(xyz, tets, weights)
    Aoff = assemble_offdiag(n, tets, Ke)
    diag = -row_sums(Aoff)
    A = (Aoff + sp.diags(diag)).tocsr()
    A.sort_indices()
    return A, Aoff


def assemble_diagonal_direct(xyz, tets):
    """sum_e K_e[a, a] assembled directly (used only to pin the row-sum form)."""
    n = xyz.shape[0]
    Ke = element_stiffness(xyz, tets)
    out = np.zeros(n)
    for a in range(4):
        np.add.at(out, tets[:, a], Ke[:, a, a])
    return out


def assemble_mass(xyz, tets):
    """Consistent mass matrix M of eq. Ax=b: M_ij = int N_i N_j."""
    n = xyz.shape[0]
    Me = element_mass(xyz, tets)
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    M = sp.csr_matrix((Me.reshape(-1), (rows, cols)), shape=(n, n))
    M.sum_duplicates()
    return M


def top_surface_mass(xyz, tri):
    """Robin term of the free-surface condition (Section 2).  Backward Euler
    applied to the kinematic condition turns the top condition into
    d phi/dn + alpha phi = 0 with alpha = (n.k)/(g dt^2) >= 0 (the printed
    form has its sign garbled; this is the reading that gives an SPD
    problem).  Its weak form adds alpha int_top (n.k) phi psi dS, and
    (n.k) dS is the horizontally projected area element, so the term is the
    P1 mass matrix of the top triangles projected onto (x, y).

    tri: top triangles (sorted vertex triples in ascending order).  Returns
    (Moff, L): Moff the off-diagonal part on the triangles' edges, each value
    a left-to-right sum of area/12 over the triangles holding the edge in
    ascending order (symmetric CSR, sorted indices, no diagonal, shape n x n
    with n = number of nodes); L_i the left-to-right sum of area/3 over the
    triangles holding node i (the row sums of the mass matrix)."""
    n = xyz.shape[0]
    tri = np.asarray(tri, dtype=np.int64)
    x1, y1 = xyz[tri[:, 0], 0], xyz[tri[:, 0], 1]
    x2, y2 = xyz[tri[:, 1], 0], xyz[tri[:, 1], 1]
    x3, y3 = xyz[tri[:, 2], 0], xyz[tri[:, 2], 1]
    area = 0.5 * np.abs((x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1))
    pairs = ((0, 1), (0, 2), (1, 2))
    lo = np.stack([np.minimum(tri[:, a], tri[:, b]) for a, b in pairs], axis=1)
    hi = np.stack([np.maximum(tri[:, a], tri[:, b]) for a, b in pairs], axis=1)
    key = (lo * n + hi).ravel()
    ukey, inv = np.unique(key, return_inverse=True)
    w = _sequential_sum_by_key(inv, np.repeat(area / 12.0, 3), ukey.size)
    ei, ej = ukey // n, ukey % n
    Moff = sp.csr_matrix((np.concatenate([w, w]), (np.concatenate([ei, ej]), np.concatenate([ej, ei]))),
                         shape=(n, n))
    Moff.sort_indices()
    L = _sequential_sum_by_key(tri.ravel(), np.repeat(area / 3.0, 3), n)
    return Moff, L


def add_robin(Aoff, Moff, L, alpha):
    """A + alpha M_top in difference form: off-diagonals a_ij + alpha m_ij on
    the pattern of Aoff (which contains every top edge), and the deficit
    alpha L_i that the Robin term adds (M_top applied to a constant)."""
    Aoff = Aoff.tocsr()
    M = Moff.tocsr()
    rows = np.repeat(np.arange(Aoff.shape[0]), np.diff(Aoff.indptr))
    m_on = np.asarray(M[rows, Aoff.indices]).ravel()
    if abs(M.sum() - m_on.sum()) > 1e-12 * abs(M.sum()):
        raise ValueError("a top edge is not a mesh edge")
    out = Aoff.copy()
    out.data = Aoff.data + alpha * m_on
    return out, alpha * L


def pin_node(xyz, top):
    """Point condition phi(x_0) = 0 with x_0 on the top surface (eq. point
    condition).  Reading: the top node closest to the origin corner, ties to
    the smallest index.  Pinned against the box's known corner node and a
    brute-force search (tests/test_oracle_pins.py)."""
    idx = np.nonzero(top)[0]
    d2 = xyz[idx, 0] ** 2 + xyz[idx, 1] ** 2 + xyz[idx, 2] ** 2
    return int(idx[np.argmin(d2)])


def dirichlet_set(xyz, top, mode, pin=-1):
    """Nodes whose value is fixed to zero.

    mode 'N': the Neumann problem with the point condition (Section 3,
    eq. point condition) -- only x_0 is fixed.
    mode 'D': Dirichlet condition on the whole top surface (eq. dirichlet).
    mode 'R': the Robin condition of the free surface (see top_surface_mass)
    -- nothing is fixed.
    """
    n = xyz.shape[0]
    D = np.zeros(n, dtype=bool)
    if mode == "N":
        D[pin if pin >= 0 else pin_node(xyz, top)] = True
    elif mode == "D":
        D[top] = True
    elif mode != "R":
        raise ValueError(mode)
    return D


def reduce_to_unknowns(Aoff, D):
    """Restriction of A to the free nodes U, in difference form.

    For i in U: (A_UU x)_i = sum_{j in U, j != i} a_ij (x_j - x_i) + d_i x_i
    with the deficit d_i = -sum_{j in D} a_ij (ascending j).  Because
    a_ii = -sum_{j != i} a_ij, this is exactly the row of A_UU.
    Returns (U index array, Aoff_UU CSR, d)."""
    U = np.nonzero(~D)[0]
    Aoff = Aoff.tocsr()
    rows = np.repeat(np.arange(Aoff.shape[0]), np.diff(Aoff.indptr))
    mask = D[Aoff.indices]
    d_full = -_sequential_sum_by_key(rows[mask], Aoff.data[mask], Aoff.shape[0])
    Auu = Aoff[U][:, U].tocsr()
    Auu.sort_indices()
    return U, Auu, d_full[U] + 0.0


def apply_difference_form(Aoff, d, x):
    """y_i = sum_{j != i} a_ij (x_j - x_i) + d_i x_i (the row of A_UU)."""
    rows = np.repeat(np.arange(Aoff.shape[0]), np.diff(Aoff.indptr))
    contrib = Aoff.data * (x[Aoff.indices] - x[rows])
    return np.bincount(rows, weights=contrib, minlength=Aoff.shape[0]) + d * x


def residual_extended(Aoff, d, b, hi, lo):
    """b - A_UU (hi + lo) for a solution held as the unevaluated sum of two
    doubles, in the difference form, evaluated in numpy.longdouble (x87
    extended precision, 64-bit significand) and rounded to FP64 once.

    Not part of the paper: Section 6 attributes the accuracy floor of its
    FP64 runs to round-off growing with the condition number; evaluating the
    restart residual of PCG this way removes that floor (see pcg.py)."""
    L = np.longdouble
    if np.finfo(L).nmant < 63:
        raise RuntimeError("numpy.longdouble is not an extended-precision type on this platform")
    h = np.asarray(hi, dtype=L)
    l = np.asarray(lo, dtype=L)
    rows = np.repeat(np.arange(Aoff.shape[0]), np.diff(Aoff.indptr))
    # the differences are taken part by part: for neighbouring values the
    # difference of the high parts is exact, so no rounding of hi + lo itself
    # enters (it would be amplified by the large vertical couplings)
    diff = (h[Aoff.indices] - h[rows]) + (l[Aoff.indices] - l[rows])
    acc = np.zeros(Aoff.shape[0], dtype=L)
    np.add.at(acc, rows, Aoff.data.astype(L) * diff)
    dl = np.asarray(d, dtype=L)
    return (np.asarray(b, dtype=L) - (acc + (dl * h + dl * l))).astype(np.float64)


def diagonal_of(Aoff, d):
    """a_ii = d_i - sum_{j in U} a_ij (ascending j)."""
    return d - row_sums(Aoff)


def full_matrix(Aoff, d):
    """Standard CSR form of A_UU: the off-diagonal pattern (numerical zeros
    kept) plus the diagonal a_ii = d_i - sum_j a_ij."""
    Aoff = Aoff.tocsr()
    n = Aoff.shape[0]
    rows = np.concatenate([np.repeat(np.arange(n), np.diff(Aoff.indptr)), np.arange(n)])
    cols = np.concatenate([Aoff.indices, np.arange(n)])
    vals = np.concatenate([Aoff.data, diagonal_of(Aoff, d)])
    order = np.lexsort((cols, rows))
    indptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))])
    A = sp.csr_matrix((vals[order], cols[order], indptr), shape=(n, n))
    A.has_sorted_indices = True
    return A
