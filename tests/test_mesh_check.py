"""Host-side mesh validation of the library (hl_mesh_check, also run by
hl_mesh_upload): positive orientation and conformity of a simplicial mesh
(Section 3.1, "Mesh and notation": cells that meet face to face).  Runs on
the CPU (no GPU call) through the C-ABI."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

pytestmark = pytest.mark.skipif(not os.path.exists(H.LIB_PATH), reason="libhyperlag.so not built")


def _merge(x, cells, tol=1e-12):
    """Merge coincident nodes (meshes glued from pieces)."""
    key = np.round(np.asarray(x) / tol).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    return np.asarray(x)[first], inv.reshape(-1)[np.asarray(cells)].astype(np.int32)


@pytest.mark.parametrize("make", [lambda: W.plane_wave_2d(n=5), lambda: W.rotating_cube_3d(n=3),
                                  lambda: W.impact_bar_3d(nx=6, ny=2, graded=True),
                                  lambda: W.swinging_plate_2d(n=4)])
def test_generated_meshes_are_conforming(make):
    w = make()
    assert H.mesh_check(w.dim, w.x, w.cells) == H.HL_OK


def test_refined_meshes_are_conforming():
    for w in (W.rotating_cube_3d(n=2), W.plane_wave_2d(n=3)):
        x, cells, _, _ = O.refine(w.dim, w.x, w.cells, w.nwall, w.normals, levels=1)
        assert H.mesh_check(w.dim, x, cells) == H.HL_OK


def test_hanging_node_2d():
    """Two unit squares side by side; the right one's left edge carries a
    midpoint node that the left square's edge does not have."""
    A, B, C, D = (0, 0), (1, 0), (1, 1), (0, 1)
    E, F, M = (2, 0), (2, 1), (1, 0.5)
    x = np.array([A, B, C, D, E, F, M], float)
    cells = np.array([[0, 1, 2], [0, 2, 3], [1, 4, 6], [4, 5, 6], [5, 2, 6]], np.int32)
    assert H.mesh_check(2, x, cells) == H.HL_E_NONCONFORMING
    # the same squares with the diagonal node shared: conforming
    cells_ok = np.array([[0, 1, 6], [0, 6, 2], [0, 2, 3], [1, 4, 6], [4, 5, 6], [5, 2, 6]], np.int32)
    assert H.mesh_check(2, x, cells_ok) == H.HL_OK


def test_hanging_nodes_3d():
    """A tetrahedron next to a red-refined one: the edge midpoints of the
    refined side lie on the coarse cell's face."""
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
    t1 = [0, 1, 2, 3]
    t2 = [1, 2, 3, 4]   # positively oriented, shares face (1, 2, 3)
    assert H.mesh_check(3, x, np.array([t1, t2], np.int32)) == H.HL_OK
    xr, cr, _, _ = O.refine(3, x, np.array([t2], np.int32), np.zeros(5, np.uint8), np.zeros((5, 3, 3)), 1)
    xs = np.vstack([x, xr])
    cs = np.vstack([np.array([t1], np.int32), cr + len(x)])
    xs, cs = _merge(xs, cs)
    assert H.mesh_check(3, xs, cs) == H.HL_E_NONCONFORMING


def test_face_of_three_cells_and_same_side_cells():
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.3, 0.3, 1], [0.3, 0.3, -1], [0.2, 0.2, 0.5]], float)
    above, below, above2 = [0, 1, 2, 3], [0, 2, 1, 4], [0, 1, 2, 5]
    assert H.mesh_check(3, x, np.array([above, below], np.int32)) == H.HL_OK
    # two cells on the same side of the shared face (they overlap)
    assert H.mesh_check(3, x, np.array([above, above2], np.int32)) == H.HL_E_NONCONFORMING
    # a face of three cells
    assert H.mesh_check(3, x, np.array([above, below, above2], np.int32)) == H.HL_E_NONCONFORMING


def test_cubes_meeting_along_an_edge_are_accepted():
    """Two Kuhn cubes sharing only an edge: the boundary is not a manifold
    there (four boundary faces on the edge), but the cells meet face to face
    and no node hangs."""
    x1, c1, _ = W.tet_mesh([0, 1], [0, 1], [0, 1])
    x2, c2, _ = W.tet_mesh([1, 2], [1, 2], [0, 1])
    x, cells = _merge(np.vstack([x1, x2]), np.vstack([c1, c2 + len(x1)]))
    assert H.mesh_check(3, x, cells) == H.HL_OK


def test_orientation_and_ids():
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    assert H.mesh_check(3, x, np.array([[0, 1, 2, 3]], np.int32)) == H.HL_OK
    assert H.mesh_check(3, x, np.array([[0, 2, 1, 3]], np.int32)) == H.HL_E_DEGENERATE_CELL
    flat = x.copy()
    flat[3] = [0.5, 0.5, 0.0]
    assert H.mesh_check(3, flat, np.array([[0, 1, 2, 3]], np.int32)) == H.HL_E_DEGENERATE_CELL
    assert H.mesh_check(3, x, np.array([[0, 1, 2, 4]], np.int32)) == H.HL_E_INVALID
    bad = x.copy()
    bad[1, 0] = np.nan
    assert H.mesh_check(3, bad, np.array([[0, 1, 2, 3]], np.int32)) == H.HL_E_INVALID
    assert H.mesh_check(4, x, np.array([[0, 1, 2, 3]], np.int32)) == H.HL_E_INVALID
    assert H.mesh_check(2, np.zeros((0, 2)), np.zeros((0, 3), np.int32)) == H.HL_OK
