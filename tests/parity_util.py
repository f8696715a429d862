"""Helpers shared by the GPU parity tests: run the HIP path and the oracle
on the same seeded input and compare them field by field."""
import math

import numpy as np

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H

FIELDS = ("x", "vhat", "tau", "v", "e", "B")


def err(a, b):
    """Normwise relative error max|a - b| / max|b| (0 if both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if b.size else 0.0
    if den == 0.0:
        return num
    return num / den


def oracle_state(st):
    return O.State(st["x"], st["vhat"], st["tau"], st["v"], st["e"], st["B"])


def gpu_params(w, detect=True, cascade=2):
    return H.default_params(w.dim, detect=detect, c_cfl=w.c_cfl, cascade=cascade)


def orc_params(w, detect=True, cascade=2):
    return O.default_params(w.c_cfl, detect=detect, cascade=cascade)


def pair(w, detect=True, cascade=2, numbering=None):
    """(gpu context, oracle problem) initialised from the same workload.
    numbering: the library's internal numbering (None: its default)."""
    if numbering is None:
        ctx = H.from_workload(w, params=gpu_params(w, detect, cascade))
    else:
        ctx = H.Context(0)
        ctx.set_numbering(numbering)
        ctx.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
        ctx.init_state(w.rho0, w.mu, w.lam, w.v_cell, w.v_node, gpu_params(w, detect, cascade))
    prob = O.Problem(w, orc_params(w, detect, cascade))
    return ctx, prob


def compare_states(ctx, orc_state, vstar_orc=None):
    g = ctx.state()
    out = {f: err(g[f], getattr(orc_state, f)) for f in FIELDS}
    if vstar_orc is not None:
        out["vstar"] = err(ctx.query("vstar"), vstar_orc)
    return out


def max_err(errs):
    return max(errs.values()) if errs else 0.0


def fmt(errs):
    return ", ".join(f"{k}={v:.2e}" for k, v in errs.items())


# ---------------------------------------------------------- patches
def node_cells(cells, nn):
    """Lists of cells around every node."""
    order = np.argsort(cells.ravel(), kind="stable")
    nodes = cells.ravel()[order]
    cell_of = order // cells.shape[1]
    starts = np.searchsorted(nodes, np.arange(nn + 1))
    return starts, cell_of


def patch_around(cells, nn, seeds, rings=2):
    """Cells within `rings` node-rings of the seed cells: enough to
    reproduce a seed cell's update exactly when the cascade choice is
    replayed (its nodes' velocities need the corners of ring 1, whose
    reconstruction needs ring 2)."""
    starts, cell_of = node_cells(cells, nn)
    sel = set(int(s) for s in seeds)
    frontier = set(sel)
    for _ in range(rings):
        nxt = set()
        for c in frontier:
            for p in cells[c]:
                for j in cell_of[starts[p]:starts[p + 1]]:
                    j = int(j)
                    if j not in sel:
                        nxt.add(j)
        sel |= nxt
        frontier = nxt
    return np.array(sorted(sel), dtype=np.int64)


def submesh(w, cell_ids):
    """Workload restricted to `cell_ids` (nodes renumbered)."""
    import copy
    sub = copy.copy(w)
    cells = w.cells[cell_ids]
    nodes, inv = np.unique(cells.ravel(), return_inverse=True)
    sub.cells = inv.reshape(cells.shape).astype(np.int32)
    sub.x = w.x[nodes]
    sub.nwall = w.nwall[nodes]
    sub.normals = w.normals[nodes]
    sub.rho0 = w.rho0[cell_ids]
    sub.mu = w.mu[cell_ids]
    sub.lam = w.lam[cell_ids]
    sub.v_cell = w.v_cell[cell_ids]
    sub.v_node = w.v_node[nodes]
    return sub, nodes


def relerr_scalar(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def close(a, b, tol):
    return err(a, b) <= tol or (np.abs(np.asarray(a) - np.asarray(b)).max() <= tol * 1e-300)


def isclose_rel(a, b, tol):
    return math.isclose(a, b, rel_tol=tol, abs_tol=0.0)
