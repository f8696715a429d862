"""Seeded synthetic workloads: simplicial meshes, wall constraints, material
fields and initial velocities.

This module only *generates inputs*.  It holds none of the scheme's
arithmetic (no geometry of the method, no stress, no fluxes): both the
HIP library and the CPU oracle receive exactly the arrays built here.

Mesh recipes (all seeded with numpy PCG64; jitter drawn node-major in the
node numbering order, one uniform draw per axis):

* 2D: a structured ``nx x ny`` grid of quads, each split on its
  (i,j)-(i+1,j+1) diagonal into two counter-clockwise triangles.
* 3D: a structured grid of hexahedra, each split into the six Kuhn
  tetrahedra that share the (0,0,0)-(1,1,1) diagonal; tetrahedra coming
  from odd permutations have two vertices swapped so that every cell is
  positively oriented.  The Kuhn split is conforming across cubes.

Interior nodes move by ``U[-j, j] * h`` per axis; nodes on the boundary of
the box move tangentially only and box corners stay fixed, so planar walls
stay exactly planar.  With ``j <= 0.2`` (2D) or ``j <= 0.15`` (3D) no cell
can invert (a vertex can approach the opposite face by at most
``2 * j * sqrt(2) * h`` while the smallest height is ``h / sqrt(2)``).

Cells are numbered cube by cube with the *longest* axis slowest so that
a slab of cells touches a slab of nodes that is small compared with the
whole mesh (good reuse of node data in cache).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """One mesh plus material, initial velocity and wall constraints.

    Arrays follow the C-ABI conventions: ``x`` is ``[n_nodes, dim]``,
    ``cells`` is ``[n_cells, dim+1]`` int32, ``nwall`` is ``[n_nodes]``
    uint8 (number of wall constraints at the node), ``normals`` is
    ``[n_nodes, dim, dim]`` (the first ``nwall[p]`` rows are unit wall
    normals), material and ``v_cell`` are per cell, ``v_node`` per node.
    """

    name: str
    dim: int
    x: np.ndarray
    cells: np.ndarray
    nwall: np.ndarray
    normals: np.ndarray
    rho0: np.ndarray
    mu: np.ndarray
    lam: np.ndarray
    v_cell: np.ndarray
    v_node: np.ndarray
    c_cfl: float
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


# ---------------------------------------------------------------- grids

def _axis_order(nseg):
    """Axis numbering order: shortest axis fastest, longest slowest."""
    return sorted(range(len(nseg)), key=lambda a: (nseg[a], a))


def _node_grid(coords):
    """Tensor-product node grid.  Returns node positions [nn, d], the grid
    index of every node [nn, d] and a lookup array ``gid -> node id``."""
    d = len(coords)
    nseg = [len(c) - 1 for c in coords]
    order = _axis_order(nseg)              # order[0] varies fastest
    shape_slow_first = [len(coords[a]) for a in reversed(order)]
    mesh_idx = np.indices(shape_slow_first).reshape(d, -1)   # slow..fast
    gidx = np.empty((mesh_idx.shape[1], d), dtype=np.int64)
    for pos, a in enumerate(reversed(order)):
        gidx[:, a] = mesh_idx[pos]
    x = np.empty((gidx.shape[0], d), dtype=np.float64)
    for a in range(d):
        x[:, a] = np.asarray(coords[a], dtype=np.float64)[gidx[:, a]]
    lookup = np.empty([len(c) for c in coords], dtype=np.int64)
    lookup[tuple(gidx[:, a] for a in range(d))] = np.arange(gidx.shape[0])
    return x, gidx, lookup


def _local_spacing(c):
    """Per-node spacing used to scale the jitter: the smaller of the two
    adjacent segment lengths."""
    c = np.asarray(c, dtype=np.float64)
    seg = np.diff(c)
    h = np.empty_like(c)
    h[0] = seg[0]
    h[-1] = seg[-1]
    h[1:-1] = np.minimum(seg[:-1], seg[1:])
    return h


def _jitter(x, gidx, coords, jitter, seed):
    if jitter <= 0.0:
        return x
    rng = np.random.Generator(np.random.PCG64(seed))
    d = x.shape[1]
    u = rng.uniform(-1.0, 1.0, size=x.shape)
    out = x.copy()
    for a in range(d):
        n = len(coords[a])
        h = _local_spacing(coords[a])[gidx[:, a]]
        interior = (gidx[:, a] > 0) & (gidx[:, a] < n - 1)
        out[:, a] += np.where(interior, jitter * h * u[:, a], 0.0)
    return out


def tri_mesh(xs, ys, jitter=0.0, seed=0):
    """Structured triangle mesh on the tensor grid ``xs x ys``."""
    coords = [np.asarray(xs, float), np.asarray(ys, float)]
    x, gidx, lk = _node_grid(coords)
    nseg = [len(c) - 1 for c in coords]
    order = _axis_order(nseg)
    # cells: quads numbered with the same axis order as nodes
    shape_slow_first = [nseg[a] for a in reversed(order)]
    q = np.indices(shape_slow_first).reshape(2, -1)
    qi = np.empty((q.shape[1], 2), dtype=np.int64)
    for pos, a in enumerate(reversed(order)):
        qi[:, a] = q[pos]
    i, j = qi[:, 0], qi[:, 1]
    n00 = lk[i, j]
    n10 = lk[i + 1, j]
    n11 = lk[i + 1, j + 1]
    n01 = lk[i, j + 1]
    tri = np.empty((qi.shape[0], 2, 3), dtype=np.int64)
    tri[:, 0] = np.stack([n00, n10, n11], axis=1)
    tri[:, 1] = np.stack([n00, n11, n01], axis=1)
    cells = tri.reshape(-1, 3).astype(np.int32)
    x = _jitter(x, gidx, coords, jitter, seed)
    return x, cells, gidx


_KUHN = []
for _perm in itertools.permutations(range(3)):
    _path = [(0, 0, 0)]
    _cur = [0, 0, 0]
    for _ax in _perm:
        _cur = list(_cur)
        _cur[_ax] = 1
        _path.append(tuple(_cur))
    # parity of the permutation
    _inv = sum(1 for a in range(3) for b in range(a + 1, 3) if _perm[a] > _perm[b])
    if _inv % 2 == 1:
        _path[1], _path[2] = _path[2], _path[1]
    _KUHN.append(_path)


def tet_mesh(xs, ys, zs, jitter=0.0, seed=0):
    """Structured Kuhn tetrahedral mesh on the tensor grid ``xs x ys x zs``."""
    coords = [np.asarray(xs, float), np.asarray(ys, float), np.asarray(zs, float)]
    x, gidx, lk = _node_grid(coords)
    nseg = [len(c) - 1 for c in coords]
    order = _axis_order(nseg)
    shape_slow_first = [nseg[a] for a in reversed(order)]
    q = np.indices(shape_slow_first).reshape(3, -1)
    qi = np.empty((q.shape[1], 3), dtype=np.int64)
    for pos, a in enumerate(reversed(order)):
        qi[:, a] = q[pos]
    tets = np.empty((qi.shape[0], 6, 4), dtype=np.int64)
    for t, path in enumerate(_KUHN):
        for k, (a, b, c) in enumerate(path):
            tets[:, t, k] = lk[qi[:, 0] + a, qi[:, 1] + b, qi[:, 2] + c]
    cells = tets.reshape(-1, 4).astype(np.int32)
    x = _jitter(x, gidx, coords, jitter, seed)
    return x, cells, gidx


def box_walls(gidx, coords, faces):
    """Slip-wall constraints on planar box faces.

    ``faces`` lists ``(axis, side)`` pairs, side 0 = low end, 1 = high end.
    A node on k listed faces gets k unit normals (``nwall = k``)."""
    nn, d = gidx.shape
    nwall = np.zeros(nn, dtype=np.uint8)
    normals = np.zeros((nn, d, d), dtype=np.float64)
    for axis, side in faces:
        n_ax = len(coords[axis])
        on = gidx[:, axis] == (0 if side == 0 else n_ax - 1)
        idx = np.nonzero(on)[0]
        # skip if the node already has this axis as a constraint
        for p in idx:
            k = int(nwall[p])
            if any(abs(normals[p, r, axis]) == 1.0 for r in range(k)):
                continue
            normals[p, k, axis] = -1.0 if side == 0 else 1.0
            nwall[p] = k + 1
    return nwall, normals


def _vertex_mean(x, cells):
    return x[cells].mean(axis=1)


def _uniform(n, val):
    return np.full(n, float(val), dtype=np.float64)


# -------------------------------------------------------------- configs

def plane_wave_2d(n=40, jitter=0.2, amp=1e-3, seed=0, steps=100):
    """Unit square, ``n x n`` split quads, rho0=1, mu=1, lambda=2 (P-wave
    speed 2), v = (amp sin 2 pi x, 0), slip walls on all four sides."""
    xs = np.linspace(0.0, 1.0, n + 1)
    x, cells, gidx = tri_mesh(xs, xs, jitter, seed)
    nwall, normals = box_walls(gidx, [xs, xs], [(0, 0), (0, 1), (1, 0), (1, 1)])
    nc = cells.shape[0]
    xc = _vertex_mean(x, cells)
    v_cell = np.zeros((nc, 2))
    v_cell[:, 0] = amp * np.sin(2 * math.pi * xc[:, 0])
    v_node = np.zeros_like(x)
    v_node[:, 0] = amp * np.sin(2 * math.pi * x[:, 0])
    return Workload(f"plane_wave_2d_n{n}", 2, x, cells, nwall, normals,
                    _uniform(nc, 1.0), _uniform(nc, 1.0), _uniform(nc, 2.0),
                    v_cell, v_node, 0.4, steps,
                    meta=dict(amp=amp, n=n, jitter=jitter, c=2.0))


def swinging_plate_2d(n=16, jitter=0.2, seed=0, U0=5e-4, rho0=1100.0,
                      E=1.7e7, nu=0.45):
    """Swinging plate on [0,2]^2 with the divergence-free closed-form
    velocity of the paper's first 2D test (Section 4.1); slip walls."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    xs = np.linspace(0.0, 2.0, n + 1)
    x, cells, gidx = tri_mesh(xs, xs, jitter, seed)
    nwall, normals = box_walls(gidx, [xs, xs], [(0, 0), (0, 1), (1, 0), (1, 1)])
    nc = cells.shape[0]
    omega = 0.5 * math.pi * math.sqrt(2.0 * mu / rho0)

    def vel(p):
        s = 0.5 * math.pi
        out = np.empty_like(p)
        out[:, 0] = -omega * U0 * np.sin(s * p[:, 0]) * np.cos(s * p[:, 1])
        out[:, 1] = omega * U0 * np.cos(s * p[:, 0]) * np.sin(s * p[:, 1])
        return out

    xc = _vertex_mean(x, cells)
    return Workload(f"swinging_plate_n{n}", 2, x, cells, nwall, normals,
                    _uniform(nc, rho0), _uniform(nc, mu), _uniform(nc, lam),
                    vel(xc), vel(x), 0.4, 0,
                    meta=dict(omega=omega, U0=U0, mu=mu, lam=lam, n=n, vel=vel))


def rotating_cube_3d(n=56, jitter=0.15, seed=0, omega=0.2, steps=200):
    """[0,1]^3 Kuhn mesh, rubber-like material, rigid rotation about z plus
    a bending field v_y = 0.1 sin(pi x / 2), free surfaces."""
    xs = np.linspace(0.0, 1.0, n + 1)
    x, cells, gidx = tet_mesh(xs, xs, xs, jitter, seed)
    nn, nc = x.shape[0], cells.shape[0]

    def vel(p):
        out = np.zeros_like(p)
        out[:, 0] = -omega * (p[:, 1] - 0.5)
        out[:, 1] = omega * (p[:, 0] - 0.5) + 0.1 * np.sin(0.5 * math.pi * p[:, 0])
        return out

    xc = _vertex_mean(x, cells)
    return Workload(f"rotating_cube_n{n}", 3, x, cells,
                    np.zeros(nn, np.uint8), np.zeros((nn, 3, 3)),
                    _uniform(nc, 1100.0), _uniform(nc, 8.2e5), _uniform(nc, 3.9e6),
                    vel(xc), vel(x), 0.25, steps,
                    meta=dict(n=n, jitter=jitter, omega=omega))


def impact_bar_3d(nx=240, ny=60, graded=True, jitter=0.15, seed=0, steps=500,
                  v0=-150.0):
    """Bar [0,4]x[0,1]x[0,1] hitting a rigid slip wall at x=0 with
    velocity ``v0``; aluminium-like material.  With ``graded`` the x
    spacing is h/4 on [0, 0.75] and h on [0.75, 4] (h = 1/ny), giving the
    8.1 M tet mesh at ny = 60; otherwise uniform ``nx`` segments."""
    h = 1.0 / ny
    if graded:
        nfine = int(round(0.75 / (h / 4.0)))
        ncoarse = int(round(3.25 / h))
        xs = np.concatenate([np.linspace(0.0, 0.75, nfine + 1),
                             np.linspace(0.75, 4.0, ncoarse + 1)[1:]])
    else:
        xs = np.linspace(0.0, 4.0, nx + 1)
    ys = np.linspace(0.0, 1.0, ny + 1)
    x, cells, gidx = tet_mesh(xs, ys, ys, jitter, seed)
    nwall, normals = box_walls(gidx, [xs, ys, ys], [(0, 0)])
    nn, nc = x.shape[0], cells.shape[0]
    v_cell = np.zeros((nc, 3))
    v_cell[:, 0] = v0
    v_node = np.zeros((nn, 3))
    v_node[:, 0] = v0
    return Workload(f"impact_bar_{'graded' if graded else 'uniform'}_ny{ny}", 3,
                    x, cells, nwall, normals,
                    _uniform(nc, 2700.0), _uniform(nc, 2.6e10), _uniform(nc, 5.1e10),
                    v_cell, v_node, 0.25, steps,
                    meta=dict(nx=len(xs) - 1, ny=ny, graded=graded, v0=v0))


def plane_wave_3d(n=8, jitter=0.15, amp=1e-6, seed=0):
    """Unit cube, rho0=1, mu=1, lambda=2, v = (amp sin 2 pi x, 0, 0), slip
    walls on all six faces (a standing P-wave with speed 2)."""
    xs = np.linspace(0.0, 1.0, n + 1)
    x, cells, gidx = tet_mesh(xs, xs, xs, jitter, seed)
    faces = [(a, s) for a in range(3) for s in range(2)]
    nwall, normals = box_walls(gidx, [xs, xs, xs], faces)
    nc = cells.shape[0]
    xc = _vertex_mean(x, cells)
    v_cell = np.zeros((nc, 3))
    v_cell[:, 0] = amp * np.sin(2 * math.pi * xc[:, 0])
    v_node = np.zeros_like(x)
    v_node[:, 0] = amp * np.sin(2 * math.pi * x[:, 0])
    return Workload(f"plane_wave_3d_n{n}", 3, x, cells, nwall, normals,
                    _uniform(nc, 1.0), _uniform(nc, 1.0), _uniform(nc, 2.0),
                    v_cell, v_node, 0.25, 0, meta=dict(amp=amp, n=n, c=2.0))


def plane_faces(w, axis, value, tol=1e-12):
    """Faces of ``w`` whose nodes all have coordinate ``axis`` equal to
    ``value`` (a planar side of a box mesh): (cells int32, local face
    uint8), face k being the one opposite the cell's k-th node."""
    on = np.abs(w.x[:, axis] - value) < tol
    onc = on[w.cells]
    cells, faces = [], []
    for k in range(w.dim + 1):
        m = np.all(np.delete(onc, k, axis=1), axis=1)
        idx = np.nonzero(m)[0]
        cells.append(idx)
        faces.append(np.full(len(idx), k))
    return np.concatenate(cells).astype(np.int32), np.concatenate(faces).astype(np.uint8)


def shear_modulus_field(nc, mu0=8.2e5, sigma=0.2, seed=1):
    """Per-cell shear modulus mu0 * clip(exp(sigma g), 0.5, 2), g ~ N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal(nc)
    return mu0 * np.clip(np.exp(sigma * g), 0.5, 2.0)


def identification_cube_3d(n=32, jitter=0.15, seed=0, mu_seed=1, steps=200):
    """Cube for shear-modulus identification: the rotating-cube bending
    field with rotation switched off, per-cell lognormal-clipped mu."""
    w = rotating_cube_3d(n=n, jitter=jitter, seed=seed, omega=0.0, steps=steps)
    w.mu = shear_modulus_field(w.n_cells, seed=mu_seed)
    w.name = f"identification_cube_n{n}"
    return w


def mesh_family(n_meshes=256, seed=0, nmin=5e3, nmax=2e5):
    """Batch of independent meshes: dim ~ Bernoulli(1/2), cell count
    log-uniform in [nmin, nmax], mu ~ U[0.5, 2] * 1e6, lambda = 2 mu,
    rho0 = 1000, v0 = A (sin pi y, sin pi x[, 0]), A ~ U[1e-3, 1e-1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for m in range(n_meshes):
        dim = 2 if rng.uniform() < 0.5 else 3
        target = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        mu = rng.uniform(0.5, 2.0) * 1e6
        amp = rng.uniform(1e-3, 1e-1)
        if dim == 2:
            k = max(2, int(round(math.sqrt(target / 2.0))))
            xs = np.linspace(0.0, 1.0, k + 1)
            x, cells, gidx = tri_mesh(xs, xs, 0.15, seed + 1 + m)
        else:
            k = max(2, int(round((target / 6.0) ** (1.0 / 3.0))))
            xs = np.linspace(0.0, 1.0, k + 1)
            x, cells, gidx = tet_mesh(xs, xs, xs, 0.15, seed + 1 + m)
        nn, nc = x.shape[0], cells.shape[0]

        def vel(p, amp=amp, dim=dim):
            out_v = np.zeros((p.shape[0], dim))
            out_v[:, 0] = amp * np.sin(math.pi * p[:, 1])
            out_v[:, 1] = amp * np.sin(math.pi * p[:, 0])
            return out_v

        xc = _vertex_mean(x, cells)
        out.append(Workload(f"family_{m}_{dim}d_k{k}", dim, x, cells,
                            np.zeros(nn, np.uint8), np.zeros((nn, dim, dim)),
                            _uniform(nc, 1000.0), _uniform(nc, mu), _uniform(nc, 2 * mu),
                            vel(xc), vel(x), 0.4 if dim == 2 else 0.25, 100,
                            meta=dict(k=k, amp=amp)))
    return out


def perturb_state(rng, n, scale):
    """Random perturbation helper used by tests to build general states."""
    return scale * rng.uniform(-1.0, 1.0, size=n)
