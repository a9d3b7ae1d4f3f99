"""Seeded thin-domain tetrahedral meshes of the kind the paper tests on.

The paper's own meshes (a Delaunay mesh of 57,453 roughly equispaced points
and a 99,017-point mesh clustered at the centre, Section 6) are not
available, so these generators produce stand-ins with the same character:
P1 tetrahedra filling a thin box, vertical coasts, a top surface at z = 0
(Section 2.1), unstructured in the vertical because every layer is jittered
independently (columns are broken).

Node numbering ("natural order") of the structured box is
``v = i + nx*(j + ny*k)`` with ``k = nz-1`` the top layer.  Everything here is
geometry and random numbers; no part of the solver method is computed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Kuhn (Freudenthal) split of a hexahedral cell into 6 tetrahedra along the
# v000 -> v111 diagonal: one tetrahedron per ordering of the three axes.
_AXIS_ORDERS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclass
class Mesh:
    xyz: np.ndarray          # [n, 3] float64 vertex coordinates
    tets: np.ndarray         # [T, 4] int64, positively oriented
    top: np.ndarray          # [n] bool, vertex lies on the top surface z = eta(x, y)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


def _signed_volumes(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    p0 = xyz[tets[:, 0]]
    a = xyz[tets[:, 1]] - p0
    b = xyz[tets[:, 2]] - p0
    c = xyz[tets[:, 3]] - p0
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def _floor_depth(x, y, H, bathymetry):
    if bathymetry:
        return -H * (1.0 + 0.3 * np.sin(2.0 * np.pi * x) * np.sin(2.0 * np.pi * y))
    return np.full_like(x, -H)


def _kuhn_tets(nx: int, ny: int, nz: int) -> np.ndarray:
    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    # cell-major order with i fastest, matching the vertex numbering
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()

    def vid(a, b, c):
        return (ci + a) + nx * ((cj + b) + ny * (ck + c))

    out = np.empty((ci.size, 6, 4), dtype=np.int64)
    for t, order in enumerate(_AXIS_ORDERS):
        step = [0, 0, 0]
        path = [vid(0, 0, 0)]
        for ax in order[:2]:
            step[ax] = 1
            path.append(vid(*step))
        path.append(vid(1, 1, 1))
        # odd permutations of the axes give negative orientation: swap last two
        parity = sum(1 for p in range(3) for q in range(p + 1, 3) if order[p] > order[q]) % 2
        if parity:
            path[2], path[3] = path[3], path[2]
        out[:, t, :] = np.stack(path, axis=1)
    return out.reshape(-1, 4)


def box_mesh(nx: int, ny: int, nz: int, H: float, *, bathymetry: bool = False,
             jitter: float = 0.0, seed: int = 0, repair_ratio: float = 0.05,
             max_repair_rounds: int = 20) -> Mesh:
    """Thin box [0,1]x[0,1]x[z_b, 0] on an nx*ny*nz vertex grid, 6 tets per cell.

    ``jitter`` is the half-width, in units of the grid spacing, of the uniform
    horizontal displacement applied independently to every vertex with
    0 < i < nx-1 and 0 < j < ny-1 on every layer (so vertical columns are
    broken).  Random numbers come from ``np.random.default_rng(seed)``: first
    all x displacements, then all y displacements, in natural vertex order.
    Layers are sigma levels ``z_k = z_b(x, y) * (1 - k/(nz-1))`` evaluated at
    the displaced position.  A tetrahedron whose volume falls to
    ``repair_ratio`` times its undisplaced volume or below has the
    displacement of its jittered vertices halved; this repeats for at most
    ``max_repair_rounds`` rounds.
    """
    if min(nx, ny, nz) < 2:
        raise ValueError("need at least 2 vertices per direction")
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    x0 = i * hx
    y0 = j * hy
    n = x0.size
    movable = (i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1)
    dx = np.zeros(n)
    dy = np.zeros(n)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        idx = np.nonzero(movable)[0]
        dx[idx] = rng.uniform(-jitter * hx, jitter * hx, idx.size)
        dy[idx] = rng.uniform(-jitter * hy, jitter * hy, idx.size)
    frac = 1.0 - k / (nz - 1)
    tets = _kuhn_tets(nx, ny, nz)

    def coords(scale):
        x = x0 + scale * dx
        y = y0 + scale * dy
        z = _floor_depth(x, y, H, bathymetry) * frac
        z[k == nz - 1] = 0.0
        return np.stack([x, y, z], axis=1)

    nominal = _signed_volumes(coords(np.zeros(n)), tets)
    scale = np.ones(n)
    rounds = 0
    repaired = 0
    xyz = coords(scale)
    for rounds in range(max_repair_rounds + 1):
        vol = _signed_volumes(xyz, tets)
        bad = np.nonzero(vol <= repair_ratio * nominal)[0]
        if bad.size == 0 or rounds == max_repair_rounds:
            break
        verts = np.unique(tets[bad].ravel())
        verts = verts[movable[verts]]
        repaired += bad.size
        scale[verts] *= 0.5
        xyz = coords(scale)
    vol = _signed_volumes(xyz, tets)
    if np.any(vol <= 0.0):
        raise RuntimeError("mesh generation left inverted tetrahedra")
    top = k == nz - 1
    meta = dict(kind="box", nx=nx, ny=ny, nz=nz, H=H, bathymetry=bathymetry,
                jitter=jitter, seed=seed, repaired_tets=int(repaired), repair_rounds=int(rounds))
    return Mesh(xyz=xyz, tets=tets, top=top, meta=meta)


# ----------------------------------------------------------------------------
# Multiscale graded mesh (stand-in for the paper's centre-refined Mesh B)
# ----------------------------------------------------------------------------

def _graded_spacing(r, h_min):
    return h_min * (1.0 + 9.0 * np.clip((r - 0.1) / 0.4, 0.0, 1.0))


def _graded_surface_points(h_min: float, seed: int):
    """Points in [0,1]^2 with local spacing h(r), r = distance from (0.5, 0.5).

    Boundary points are placed on the four edges at the local spacing; the
    interior is filled ring by ring around the centre so that the spacing
    grows from h_min inside the disc r < 0.1 to 10 h_min for r > 0.5.
    """
    rng = np.random.default_rng(seed)
    pts = [np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])]
    # boundary edges
    for side in range(4):
        s = [0.0]
        while True:
            t = s[-1]
            p = np.array([[t, 0.0], [1.0, t], [1.0 - t, 1.0], [0.0, 1.0 - t]][side])
            h = _graded_spacing(np.hypot(p[0] - 0.5, p[1] - 0.5), h_min)
            if t + 1.5 * h > 1.0:
                break
            s.append(t + h)
        s = np.array(s[1:])
        if s.size:
            edge = np.stack([[s, np.zeros_like(s)], [np.ones_like(s), s],
                             [1.0 - s, np.ones_like(s)], [np.zeros_like(s), 1.0 - s]][side], axis=1)
            pts.append(edge)
    # interior rings
    r = 0.0
    ring_pts = [np.array([[0.5, 0.5]])]
    r = _graded_spacing(0.0, h_min)
    rmax = np.hypot(0.5, 0.5)
    while r < rmax:
        h = _graded_spacing(r, h_min)
        m = max(6, int(round(2.0 * np.pi * r / h)))
        th = (np.arange(m) + rng.uniform(0.0, 1.0)) * (2.0 * np.pi / m)
        p = np.stack([0.5 + r * np.cos(th), 0.5 + r * np.sin(th)], axis=1)
        # keep points well inside the square (boundary points are placed separately)
        d_edge = np.minimum.reduce([p[:, 0], 1.0 - p[:, 0], p[:, 1], 1.0 - p[:, 1]])
        keep = d_edge > 0.5 * _graded_spacing(np.hypot(p[:, 0] - 0.5, p[:, 1] - 0.5), h_min)
        ring_pts.append(p[keep])
        r += h
    pts.extend(ring_pts)
    return np.concatenate(pts, axis=0)


def graded_mesh(h_min: float, H: float, *, jitter: float = 0.25, seed: int = 3,
                min_layers: int = 16, max_layers: int = 64, repair_ratio: float = 0.05,
                max_repair_rounds: int = 20) -> Mesh:
    """Multiscale thin box [0,1]^2 x [-H, 0], refined 10:1 towards a central disc.

    The surface is a 2-D Delaunay triangulation (SciPy) of graded points; each
    surface vertex carries a column of L+1 sigma levels, L = round(max_layers
    - (max_layers - min_layers) * (h/h_min - 1)/9), so the layer count goes from
    ``max_layers`` inside the disc to ``min_layers`` far from it.  The prism
    under each surface triangle is cut into tetrahedra by sweeping upward
    through its three columns, always advancing the column whose next level is
    lowest (ties: smallest vertex id); adjacent prisms make the same choices on
    their shared face, so the mesh is conforming.  Interior vertices are then
    jittered horizontally by up to ``jitter`` times the local spacing, layer by
    layer, with the same repair rule as :func:`box_mesh`.
    """
    from scipy.spatial import Delaunay

    p2 = _graded_surface_points(h_min, seed)
    tri = Delaunay(p2).simplices.astype(np.int64)
    # orient surface triangles counter-clockwise
    a, b, c = p2[tri[:, 0]], p2[tri[:, 1]], p2[tri[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    keep = np.abs(area2) > 1e-14
    tri = tri[keep]
    flip = area2[keep] < 0
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()

    ns = p2.shape[0]
    hloc = _graded_spacing(np.hypot(p2[:, 0] - 0.5, p2[:, 1] - 0.5), h_min)
    layers = np.rint(max_layers - (max_layers - min_layers) * (hloc / h_min - 1.0) / 9.0).astype(np.int64)
    layers = np.clip(layers, min_layers, max_layers)
    col_start = np.zeros(ns + 1, dtype=np.int64)
    col_start[1:] = np.cumsum(layers + 1)
    n = int(col_start[-1])
    col_of = np.repeat(np.arange(ns), layers + 1)
    lev = np.arange(n) - col_start[col_of]
    sfrac = lev / layers[col_of]             # 0 at the floor, 1 at the top

    # sweep-merge tetrahedralisation of every prism, vectorised over prisms
    nt = tri.shape[0]
    cur = np.zeros((nt, 3), dtype=np.int64)  # current level of each of the 3 columns
    L3 = layers[tri]
    total = L3.sum(axis=1)
    steps = int(total.max())
    tets = []
    for _ in range(steps):
        active = (cur < L3).any(axis=1)
        if not active.any():
            break
        nxt = np.where(cur < L3, (cur + 1) / L3, np.inf)
        # tie-break on vertex id: smaller id advances first
        key_id = np.where(cur < L3, tri, np.iinfo(np.int64).max)
        order = np.argsort(key_id, axis=1, kind="stable")
        nxt_sorted = np.take_along_axis(nxt, order, axis=1)
        pick_sorted = np.argmin(nxt_sorted, axis=1)
        pick = order[np.arange(nt), pick_sorted]
        rows = np.nonzero(active)[0]
        base = col_start[tri[rows]] + cur[rows]
        pk = pick[rows]
        new_v = col_start[tri[rows, pk]] + cur[rows, pk] + 1
        tets.append(np.concatenate([base, new_v[:, None]], axis=1))
        cur[rows, pk] += 1
    tets = np.concatenate(tets, axis=0)

    boundary2 = (p2[:, 0] <= 0.0) | (p2[:, 0] >= 1.0) | (p2[:, 1] <= 0.0) | (p2[:, 1] >= 1.0)
    movable = ~boundary2[col_of]
    rng = np.random.default_rng(seed + 1)
    idx = np.nonzero(movable)[0]
    dx = np.zeros(n)
    dy = np.zeros(n)
    hv = hloc[col_of]
    dx[idx] = rng.uniform(-1.0, 1.0, idx.size) * jitter * hv[idx]
    dy[idx] = rng.uniform(-1.0, 1.0, idx.size) * jitter * hv[idx]
    top = lev == layers[col_of]

    def coords(scale):
        x = p2[col_of, 0] + scale * dx
        y = p2[col_of, 1] + scale * dy
        z = -H * (1.0 - sfrac)
        return np.stack([x, y, z], axis=1)

    xyz0 = coords(np.zeros(n))
    vol0 = _signed_volumes(xyz0, tets)
    neg = vol0 < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    nominal = np.abs(vol0)
    scale = np.ones(n)
    xyz = coords(scale)
    repaired = 0
    rounds = 0
    for rounds in range(max_repair_rounds + 1):
        vol = _signed_volumes(xyz, tets)
        bad = np.nonzero(vol <= repair_ratio * nominal)[0]
        if bad.size == 0 or rounds == max_repair_rounds:
            break
        verts = np.unique(tets[bad].ravel())
        verts = verts[movable[verts]]
        repaired += bad.size
        scale[verts] *= 0.5
        xyz = coords(scale)
    if np.any(_signed_volumes(xyz, tets) <= 0.0):
        raise RuntimeError("graded mesh generation left inverted tetrahedra")
    meta = dict(kind="graded", h_min=h_min, H=H, jitter=jitter, seed=seed,
                surface_points=int(ns), repaired_tets=int(repaired), repair_rounds=int(rounds))
    return Mesh(xyz=xyz, tets=tets, top=top, meta=meta)
