"""Pins of the oracle's conforming red refinement (Section 3.9: the local
1 -> 8 split of the tetrahedra of a coarse mesh; 1 -> 4 for triangles).

Fixed by geometry and topology, not by the refinement's own formulas:
children fill their parent exactly (volumes sum to it, the corner children
are the parent scaled by 1/2 about a vertex), all are positively oriented;
the refined mesh is conforming (every face has at most two cells, the
boundary faces are the parent's split in 4 / edges split in 2) and keeps
the Euler characteristic of a ball; new nodes sit at the edge midpoints,
all distinct; the octahedron is split along its shortest diagonal; box
walls pass to the midpoints on the box faces; two levels equal one level
applied twice.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W


def _measure(X):
    d = X.shape[1]
    return np.linalg.det(X[1:] - X[0]) / (6.0 if d == 3 else 2.0)


def _faces(cells):
    cnt = {}
    for c in cells:
        for f in itertools.combinations(sorted(int(k) for k in c), len(c) - 1):
            cnt[f] = cnt.get(f, 0) + 1
    return cnt


def _edges(cells):
    return {e for c in cells for e in itertools.combinations(sorted(int(k) for k in c), 2)}


CASES = {
    "cube": lambda: W.rotating_cube_3d(n=2, seed=3),
    "bar": lambda: W.impact_bar_3d(nx=4, ny=2, graded=False, seed=5),
    "square": lambda: W.plane_wave_2d(n=4, seed=2),
}


def _ref(w, levels=1):
    return O.refine(w.dim, w.x, w.cells, w.nwall, w.normals, levels)


@pytest.mark.parametrize("case", list(CASES))
def test_children_fill_the_parent(case):
    w = CASES[case]()
    x, cells, _, _ = _ref(w)
    d = w.dim
    nch = 8 if d == 3 else 4
    assert cells.shape == (w.n_cells * nch, d + 1)
    for c in range(w.n_cells):
        V = _measure(w.x[w.cells[c]])
        ch = [_measure(x[cells[nch * c + j]]) for j in range(nch)]
        assert min(ch) > 0
        assert sum(ch) == pytest.approx(V, rel=1e-13)
        for j in range(d + 1):          # corner children: scaled by 1/2
            assert ch[j] == pytest.approx(V / 2 ** d, rel=1e-13)


@pytest.mark.parametrize("case", list(CASES))
def test_refined_mesh_is_conforming(case):
    w = CASES[case]()
    x, cells, _, _ = _ref(w)
    f0, f1 = _faces(w.cells), _faces(cells)
    assert max(f1.values()) == 2
    b0 = sum(v == 1 for v in f0.values())
    b1 = sum(v == 1 for v in f1.values())
    assert b1 == (4 if w.dim == 3 else 2) * b0
    # Euler characteristic of a ball: V - E + F - C = 1 (3D), V - E + F = 1 (2D)
    E = len(_edges(cells))
    chi = len(x) - E + (len(f1) - len(cells) if w.dim == 3 else len(cells))
    assert chi == 1


@pytest.mark.parametrize("case", list(CASES))
def test_new_nodes_are_the_edge_midpoints(case):
    w = CASES[case]()
    x, cells, _, _ = _ref(w)
    edges = sorted(_edges(w.cells))
    assert len(x) == w.n_nodes + len(edges)
    assert np.array_equal(x[:w.n_nodes], w.x)
    mids = np.array([0.5 * (w.x[p] + w.x[q]) for p, q in edges])
    assert np.array_equal(x[w.n_nodes:], mids)
    assert len(np.unique(np.round(x, 12), axis=0)) == len(x)


@pytest.mark.parametrize("case", ["cube", "bar"])
def test_octahedron_split_along_the_shortest_diagonal(case):
    w = CASES[case]()
    x, cells, _, _ = _ref(w)
    for c in range(w.n_cells):
        octa = cells[8 * c + 4: 8 * c + 8]
        shared = set(octa[0])
        for t in octa[1:]:
            shared &= set(t)
        assert len(shared) == 2               # the four share the diagonal
        mids = set(np.unique(octa))
        assert len(mids) == 6 and all(k >= w.n_nodes for k in mids)
        a, b = sorted(shared)
        others = sorted(mids - shared)
        dl = np.sum((x[a] - x[b]) ** 2)
        # the opposite pairs of the octahedron are the other diagonals
        opp = [(p, q) for p, q in itertools.combinations(others, 2)
               if not any({p, q} <= set(t) for t in octa)]
        assert len(opp) == 2
        for p, q in opp:
            assert dl <= np.sum((x[p] - x[q]) ** 2) * (1 + 1e-12)


def test_walls_pass_to_midpoints_on_the_walls():
    w = W.rotating_cube_3d(n=2, seed=3)
    w.nwall = np.zeros(w.n_nodes, np.uint8)
    w.normals = np.zeros((w.n_nodes, 3, 3))
    for p in range(w.n_nodes):
        for ax in range(3):
            if abs(w.x[p, ax]) < 1e-12:
                w.normals[p, w.nwall[p], ax] = 1.0
                w.nwall[p] += 1
    x, cells, nwall, normals = _ref(w)
    for p in range(w.n_nodes, len(x)):
        on = [ax for ax in range(3) if abs(x[p, ax]) < 1e-12]
        assert nwall[p] == len(on)
        got = sorted(int(np.argmax(np.abs(normals[p, r]))) for r in range(nwall[p]))
        assert got == on


def test_two_levels_equal_one_level_twice():
    w = CASES["bar"]()
    a = _ref(w, 2)
    x1, c1, n1, r1 = _ref(w, 1)
    b = O.refine(3, x1, c1, n1, r1, 1)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
