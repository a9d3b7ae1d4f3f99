"""Pins of the multiscale graded mesh (the centre-refined stand-in for the
paper's Mesh B): a conforming positively oriented P1 mesh of the thin box,
whose top surface covers the unit square and whose layer count follows the
grading."""
import numpy as np
import pytest

from inputs import graded_mesh
from oracle import extrap, fem


@pytest.fixture(scope="module")
def mesh():
    return graded_mesh(1 / 60, 1e-3, jitter=0.25, seed=3)


def test_positive_volumes_and_total_volume(mesh):
    _, det = fem.element_geometry(mesh.xyz, mesh.tets)
    assert det.min() > 0
    assert abs(det.sum() / 6.0 - 1e-3) < 1e-15


def test_conforming_faces(mesh):
    t = mesh.tets
    faces = np.sort(np.concatenate([t[:, [0, 1, 2]], t[:, [0, 1, 3]], t[:, [0, 2, 3]], t[:, [1, 2, 3]]]), axis=1)
    uniq, count = np.unique(faces, axis=0, return_counts=True)
    assert count.max() == 2
    # faces used once lie on the box boundary
    bnd = uniq[count == 1]
    p = mesh.xyz[bnd]
    on = ((np.abs(p[:, :, 0]) < 1e-12).all(1) | (np.abs(p[:, :, 0] - 1) < 1e-12).all(1) |
          (np.abs(p[:, :, 1]) < 1e-12).all(1) | (np.abs(p[:, :, 1] - 1) < 1e-12).all(1) |
          (np.abs(p[:, :, 2]) < 1e-15).all(1) | (np.abs(p[:, :, 2] + 1e-3) < 1e-15).all(1))
    assert on.all()


def test_top_surface_covers_unit_square(mesh):
    tri = extrap.top_triangles(mesh.tets, mesh.top)
    p = mesh.xyz[tri][:, :, :2]
    area = 0.5 * np.abs((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) -
                        (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0]))
    assert abs(area.sum() - 1.0) < 1e-12


def test_layers_follow_grading(mesh):
    # 64 layers under the refined disc, 16 far from it
    top = np.nonzero(mesh.top)[0]
    r = np.hypot(mesh.xyz[top, 0] - 0.5, mesh.xyz[top, 1] - 0.5)
    # count nodes per column via unjittered column id: columns are contiguous in the numbering
    n_per_col = np.diff(np.concatenate([[-1], top]))
    assert n_per_col[r < 0.09].min() == 65
    assert n_per_col[r > 0.55].max() == 17
