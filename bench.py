#!/usr/bin/env python3
"""Throughput of the ADER-MOOD Lagrangian step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Times exactly K steps of the whole hot path (reconstruction, predictor,
nodal solve, cell update, MOOD detection and first-order recompute until no
new flag, CFL reduction) on synthetic input already resident in HBM, and
prints ONE JSON line.  The default workload is the 8.1 M-tetrahedron graded
impact bar.  Kernel durations come from HIP events recorded on the stream
the kernels run on, over the timed region; the CPU baseline is the FP64
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 cell-updates/s per Lagrangian step; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector peak: 256 CUs x 128 lanes x 2 flop (FMA) x 2.4 GHz
# algorithmic FP64 work of one cell-update (hand count of the method's
# arithmetic: geometry twice, least squares in node-aggregate form,
# predictor with the chain rule, corner matrices, node solve, update with
# the Crank-Nicolson solve, stress and detection), 3D and 2D
ALG_FLOP_PER_CELL = {3: 4600.0, 2: 1700.0}
PROFILED = ("pack", "node_agg", "predict", "node_solve", "update", "mood_sparse", "reduce")


def workloads():
    from paper_2104_02139_amd import workloads as W
    return {
        "impact_bar_graded_8.1M": lambda: W.impact_bar_3d(ny=60, graded=True),
        "impact_bar_5.2M": lambda: W.impact_bar_3d(nx=240, ny=60, graded=False),
        "rotating_cube_1.05M": lambda: W.rotating_cube_3d(n=56),
        "plane_wave_2d_3200": lambda: W.plane_wave_2d(n=40),
    }


def kernel_bytes(dim, nc, nn):
    """Bytes one launch of each stage kernel must move as built: every input
    it reads once, every output once (FP64 = 8 B, int32 = 4 B, flags 1 B),
    the staged design's intermediates (node aggregates, corner records,
    gather records) included.  Reported beside the roofline, not in it."""
    d = dim
    nv = d + 1
    ncor = nv * nc
    nB = 6 if d == 3 else 3
    nW = 1 + d + nB
    nms = 6 if d == 3 else 3
    cw = nms + d
    na = 1 + d + nms + nW + d * nW + 2
    csr = 4 * (nn + 1) + 4 * ncor
    return {
        "pack": 4 * ncor + 8 * d * nn + 8 * nW * nc + 8 * (nW + d) * nc,
        "node_agg": csr + 8 * d * nn + 8 * (nW + d) * nc + 8 * na * nn,
        "predict": 4 * ncor + 8 * d * nn + 8 * nW * nc + 24 * nc + nc + 8 * na * nn + 8 * cw * ncor,
        "node_solve": csr + 8 * cw * ncor + nn + 16 * d * nn + 24 * d * nn,
        "update": (4 * ncor + 40 * d * nn + 8 * cw * ncor + 8 * (nW + 1) * nc + 32 * nc + nc
                   + 16 * nn + 8 * (nW + 1) * nc + nc + 16 * nc + 8 * (nW + d) * nc),
    }


def step_alg_bytes(dim, nc, nn):
    """Algorithmic bytes of a whole step: cell state (tau, v, e, B) in and
    out, the cell mass, the cell -> node and node -> corner connectivity,
    node positions and carried velocities in and out, flags, each once
    (about 235 B per cell-update in 3D on a Kuhn mesh, 177 B in 2D)."""
    d = dim
    nB = 6 if d == 3 else 3
    cell_state = 1 + d + 1 + nB
    return (2 * 8 * cell_state * nc + 8 * nc + 4 * (d + 1) * nc
            + 4 * (nn + 1) + 4 * (d + 1) * nc + 2 * 2 * 8 * d * nn + nc + nn)


def kernel_source_hash():
    h = hashlib.sha1()
    for f in ("hl_kernels.hip", "hl_device.h"):
        with open(os.path.join(ROOT, "paper_2104_02139_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def read_traffic(kernel, workload):
    """HBM traffic of `kernel` from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha1") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_stage_traffic(workload):
    """Measured HBM bytes (read + written) of one launch of each stage
    kernel of the step, from the same committed counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_predict_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha1") != kernel_source_hash():
        return None
    try:
        out = {"predict": float(vals["hbm_bytes_per_launch"])}
        for k in ("node_agg", "node_solve", "update"):
            out[k] = float(vals[f"hbm_bytes_per_launch_{k}"])
        return out
    except (KeyError, ValueError):
        return None


def read_valu(kernel, workload):
    """FP64 flop of one launch of `kernel` from the committed rocprofv3
    VALU counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha1") != kernel_source_hash():
        return None
    try:
        return float(vals[f"fp64_flop_per_launch_{kernel}"])
    except (KeyError, ValueError):
        return None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(name, budget_s=12.0):
    """The oracle as it stands on a bounded sample of the workload (the same
    mesh family at a reduced resolution, steps from t = 0): its serial
    build on one core, and its OpenMP build (threads over output cells and
    nodes, bitwise the serial results) on every core the process may use."""
    from oracle import oracle as O
    from paper_2104_02139_amd import workloads as W
    if name.startswith("impact_bar"):
        w = W.impact_bar_3d(ny=16, graded=True)
        sample = "graded impact bar at ny=16 (%d tets), steps from t=0" % w.n_cells
    elif name.startswith("rotating_cube"):
        w = W.rotating_cube_3d(n=24)
        sample = "rotating cube n=24 (%d tets), steps from t=0" % w.n_cells
    else:
        w = W.plane_wave_2d(n=40)
        sample = "2D plane wave 40x40 (%d triangles), steps from t=0" % w.n_cells
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)

    def run(threads):
        O.use_threads(threads)
        try:
            prob = O.Problem(w)
            dt = prob.initial_dt()
            t0 = time.perf_counter()
            steps = 0
            while True:
                _, _, _, info = prob.step(dt)
                dt = info.dt_next
                steps += 1
                if time.perf_counter() - t0 > budget_s or steps >= 200:
                    break
            return steps, time.perf_counter() - t0
        finally:
            O.use_threads(False)

    s1, e1 = run(False)
    os.environ.setdefault("OMP_NUM_THREADS", str(ncores))
    threads = int(os.environ["OMP_NUM_THREADS"])
    sn, en = run(True)
    return {"value": w.n_cells * sn / en, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle", "sample": f"{sample}; OpenMP build, {threads} threads: {sn} steps in {en:.1f} s",
            "one_core": {"value": w.n_cells * s1 / e1, "cores": 1,
                         "sample": f"{sample}; serial build: {s1} steps in {e1:.1f} s"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def batch_measure(steps=100, warmup=10, seq_steps=10, n_meshes=256):
    """Many independent meshes (a seeded mix of 2D and 3D, log-uniform
    sizes in [5e3, 2e5] cells), per-mesh CFL dt: one batched context per
    dimension, the two stepped as a group (hl_group_step: one launch per
    stage, MOOD pass and reduction for the whole family, the step captured
    in a hipGraph), against the two contexts stepped one after the other
    and against the meshes stepped one after another on the same stream.
    Every run starts from t = 0 and times `steps` steps after `warmup`
    untimed ones (the first steps, where the relaxed DMP on rho0 = 1000
    flags most cells, stay out of the timed window)."""
    import torch
    from paper_2104_02139_amd import hyperlag as H
    from paper_2104_02139_amd import workloads as W
    ws = W.mesh_family(n_meshes)
    total = sum(w.n_cells for w in ws)
    stream = torch.cuda.current_stream()
    fam = [[w for w in ws if w.dim == d] for d in (2, 3)]
    bctx = [H.from_workloads(f, stream=stream) for f in fam]
    for c in bctx:
        c.use_graph(True, 6)
    grp = H.Group(bctx[0], bctx[1])
    grp.use_graph(True, 6)

    def restart():
        for c, f in zip(bctx, fam):
            H.init_from_workloads(c, f)
            c.compute_dt()

    def timed(step_once):
        restart()
        for _ in range(warmup):
            step_once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step_once()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    tg = timed(lambda: grp.step(info=False))
    i2, i3 = grp.step()
    mood = {"first_order_frac_2d": i2["n_p0"] / max(1, bctx[0].n_cells),
            "first_order_frac_3d": i3["n_p0"] / max(1, bctx[1].n_cells),
            "mood_iters_2d": i2["mood_iters"], "mood_iters_3d": i3["mood_iters"]}
    tb = timed(lambda: [c.step_batch(None, info=False) for c in bctx])
    grp.close()
    del bctx
    singles = [H.from_workload(w, stream=stream) for w in ws]
    for c in singles:
        c.compute_dt()
    for _ in range(2):
        for c in singles:
            c.step(0.0, info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(seq_steps):
        for c in singles:
            c.step(0.0, info=False)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / seq_steps
    return {"workload": f"mesh_family_{n_meshes}", "n_meshes": n_meshes, "n_cells_total": total,
            "n_2d": len(fam[0]), "n_3d": len(fam[1]), "steps": steps, "warmup": warmup,
            "grouped_cell_updates_per_s": total * steps / tg,
            "grouped_ms_per_step": 1e3 * tg / steps,
            "two_contexts_cell_updates_per_s": total * steps / tb,
            "sequential_cell_updates_per_s": total / ts,
            "sequential_steps": seq_steps,
            "speedup": ts / (tg / steps), "after_timed_steps": mood}


def jelly_material(w):
    """The droplet test's material (Section 4: rho0 = 1020, mu = 85,
    stiffened gas gamma = 2.2, p_inf = 1e6) on the workload's mesh, hitting
    its wall at 3 m/s."""
    import copy
    import numpy as np
    g = copy.copy(w)
    g.rho0 = np.full(w.n_cells, 1020.0)
    g.mu = np.full(w.n_cells, 85.0)
    g.v_cell = w.v_cell * (3.0 / np.abs(w.v_cell).max())
    g.v_node = w.v_node * (3.0 / np.abs(w.v_node).max())
    return g


def variant_measure(ctx, w, steps, warmup, graph, name, setup=None, **params):
    """The same workload from t = 0 with other scheme parameters -- the
    three-level cascade P1 -> P1 with the Barth-Jespersen limiter -> P0
    (Section 3.5), another member of the shear energy family (eq.
    familiy_energies) -- or with boundary conditions added by ``setup(ctx)``
    (Section 3.8: loads, contact), which must undo them when called with
    ``None``."""
    import torch
    from paper_2104_02139_amd import hyperlag as H
    ctx.init_state(w.rho0, w.mu, w.lam, w.v_cell, w.v_node,
                   H.default_params(w.dim, c_cfl=w.c_cfl, **params))
    if setup:
        setup(ctx)
    ctx.use_graph(graph, 6)
    lim, p0, it, tr, clip = [], [], [], [], 0
    for _ in range(warmup):
        inf = ctx.step(0.0, info=True)
        lim.append(inf["n_limited"])
        p0.append(inf["n_p0"])
        it.append(inf["mood_iters"])
        tr.append(inf["trials"])
        clip += inf["clipped"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(0.0, info=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    inf = ctx.step(0.0, info=True)
    lim.append(inf["n_limited"])
    p0.append(inf["n_p0"])
    it.append(inf["mood_iters"])
    out = {"variant": name, "steps": steps, "ms_per_step": 1e3 * el / steps,
           "cell_updates_per_s": w.n_cells * steps / el,
           "limited_frac_mean": sum(lim) / len(lim) / w.n_cells,
           "first_order_frac_mean": sum(p0) / len(p0) / w.n_cells,
           "mood_iters_mean": sum(it) / len(it)}
    if setup:
        out["untimed_steps_trials_mean"] = sum(tr) / max(len(tr), 1)
        out["untimed_steps_clipped"] = clip
        out["n_contact_after"] = inf["n_contact"]
        setup(None)
    return out


def bar_loads(w):
    """Boundary loads on the impact bar: the far end (x = 4) pushed at the
    impact speed (outward normal velocity -150 m/s) and a shear traction
    T13 = 10 MPa on the top face (z = 1)."""
    import numpy as np
    from paper_2104_02139_amd import workloads as W
    ce, fe = W.plane_faces(w, 0, 4.0)
    ct, ft = W.plane_faces(w, 2, 1.0)
    val = np.zeros((len(ce) + len(ct), 6))
    val[:len(ce), 0] = -150.0
    val[len(ce):, 4] = 1e7
    kind = np.concatenate([np.full(len(ce), 2), np.full(len(ct), 1)]).astype(np.uint8)
    loads = (np.concatenate([ce, ct]), np.concatenate([fe, ft]), kind, val)
    holder = {}

    def setup(ctx):
        if ctx is None:
            holder["ctx"].set_boundary_loads()
            return
        ctx.set_boundary_loads(*loads)
        holder["ctx"] = ctx
    return setup


def bar_lid(w, gap=2e-5):
    """Rigid lid above the bar: the plane z = 1 + gap (normal -z) with the
    top-face nodes as contact candidates; the bulge of the impact end
    reaches it within the first steps."""
    import numpy as np
    nodes = np.nonzero(np.abs(w.x[:, 2] - 1.0) < 1e-12)[0].astype(np.int32)
    holder = {}

    def setup(ctx):
        if ctx is None:
            holder["ctx"].set_contact()
            return
        ctx.set_contact(nodes, [0.0, 0.0, 1.0 + gap], [0.0, 0.0, -1.0])
        holder["ctx"] = ctx
    return setup


def refined_measure(w, steps, warmup, graph):
    """The paper's route to large meshes (Section 3.9): the workload's mesh
    refined once on the GPU (1 -> 8 tetrahedra, 1 -> 4 triangles), its
    cells inheriting their parent's material and velocity, then stepped
    like the main measurement.  Needs a uniform initial node velocity."""
    import numpy as np
    import torch
    from paper_2104_02139_amd import hyperlag as H
    if not np.all(w.v_node == w.v_node[:1]):
        return None
    ctx = H.Context(stream=torch.cuda.current_stream())
    ctx.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.refine(1)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    k = 8 if w.dim == 3 else 4
    rep = lambda a: np.repeat(a, k, axis=0)
    ctx.init_state(rep(w.rho0), rep(w.mu), rep(w.lam), rep(w.v_cell), np.tile(w.v_node[:1], (ctx.n_nodes, 1)),
                   H.default_params(w.dim, c_cfl=w.c_cfl))
    ctx.use_graph(graph, 6)
    it = []
    for _ in range(warmup):
        it.append(ctx.step(0.0, info=True)["mood_iters"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(0.0, info=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"n_cells": ctx.n_cells, "n_nodes": ctx.n_nodes, "refine_s_incl_upload": t_ref, "steps": steps,
           "ms_per_step": 1e3 * el / steps, "cell_updates_per_s": ctx.n_cells * steps / el,
           "mood_iters_mean": sum(it) / max(len(it), 1)}
    ctx.close()
    return out


def permuted(w, seed):
    """The workload with cells and nodes in a seeded random order, as a mesh
    from a mesher may arrive."""
    import copy
    import numpy as np
    rng = np.random.default_rng(seed)
    pc = rng.permutation(w.n_cells)
    pn = rng.permutation(w.n_nodes)
    new_of_old = np.argsort(pn)
    g = copy.copy(w)
    g.x = w.x[pn]
    g.cells = new_of_old[w.cells[pc]].astype(np.int32)
    g.nwall, g.normals, g.v_node = w.nwall[pn], w.normals[pn], w.v_node[pn]
    g.rho0, g.mu, g.lam, g.v_cell = w.rho0[pc], w.mu[pc], w.lam[pc], w.v_cell[pc]
    return g


def timed_steps(ctx, n_cells, steps, warmup, graph, report_steps=True):
    """warmup untimed steps, then `steps` timed steps as submitted in
    production; the MOOD statistics of the timed steps come from replaying
    them with reports after restoring the state they started from."""
    import torch
    ctx.use_graph(graph, 6)
    for _ in range(warmup):
        ctx.step(0.0, info=False)
    stats = None
    if report_steps:
        blob = ctx.save_state()
        p0, it, rec = [], [], []
        for _ in range(steps):
            inf = ctx.step(0.0, info=True)
            p0.append(inf["n_p0"])
            it.append(inf["mood_iters"])
            rec.append(inf["n_recomputed"])
        ctx.restore_state(blob)
        stats = {"first_order_frac_mean": sum(p0) / len(p0) / n_cells,
                 "first_order_frac_min": min(p0) / n_cells, "first_order_frac_max": max(p0) / n_cells,
                 "mood_iters_mean": sum(it) / len(it), "recomputed_per_step_mean": sum(rec) / len(rec)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(0.0, info=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"steps": steps, "ms_per_step": 1e3 * el / steps, "cell_updates_per_s": n_cells * steps / el}
    if stats:
        out.update(stats)
    return out


def workload_measure(name, w, steps, warmup, graph, numbering=None, prepare=None):
    """A workload in a context of its own, stepped from t = 0 (after
    `prepare(ctx)`, if given), timed like the headline."""
    import torch
    from paper_2104_02139_amd import hyperlag as H
    ctx = H.Context(stream=torch.cuda.current_stream())
    if numbering is not None:
        ctx.set_numbering(numbering)
    t0 = time.perf_counter()
    ctx.upload_mesh(w.dim, w.x, w.cells, w.nwall, w.normals)
    t_up = time.perf_counter() - t0
    ctx.init_state(w.rho0, w.mu, w.lam, w.v_cell, w.v_node, H.default_params(w.dim, c_cfl=w.c_cfl))
    if prepare:
        prepare(ctx)
    ctx.compute_dt()
    out = {"variant": name, "n_cells": w.n_cells, "n_nodes": w.n_nodes, "upload_s": t_up}
    out.update(timed_steps(ctx, w.n_cells, steps, warmup, graph))
    ctx.close()
    return out


def impact_noise(w, amp=1.0, xmax=0.2, seed=0):
    """Seeded velocity noise (amp m/s per component, normal) on the cells of
    the impact region x < xmax, total energy raised by the kinetic energy
    added: the relaxed DMP then flags several per cent of the cells per
    step while the noise decays."""
    import numpy as np
    xc = w.x[w.cells].mean(axis=1)
    sel = xc[:, 0] < xmax
    rng = np.random.default_rng(seed)
    v = w.v_cell.copy()
    v[sel] += amp * rng.standard_normal((int(sel.sum()), w.dim))
    e = 0.5 * np.sum(v * v, axis=1)

    def prepare(ctx):
        ctx.upload_field("v", v)
        ctx.upload_field("e", e)
    return prepare, float(sel.mean())


def adjoint_measure(n=32, steps=200, every=20):
    """Shear-modulus identification cube (32^3 Kuhn cells, lognormal mu):
    time of the checkpointed forward record, of the same steps without
    recording, and of the reverse sweep."""
    import numpy as np
    import torch
    from paper_2104_02139_amd import hyperlag as H
    from paper_2104_02139_amd import workloads as W
    w = W.identification_cube_3d(n=n, steps=steps)
    ctx = H.from_workload(w, stream=torch.cuda.current_stream())
    # one untimed step builds the launch schedules (work lists, node tiles)
    ctx.step(0.0, info=False)
    ctx.init_state(w.rho0, w.mu, w.lam, w.v_cell, w.v_node, ctx.params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(0.0, info=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ctx.init_state(w.rho0, w.mu, w.lam, w.v_cell, w.v_node, ctx.params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.forward_record(steps, every)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    g = np.random.default_rng(0).standard_normal((w.n_nodes, w.dim))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gmu, _, _ = ctx.adjoint_run(g)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    return {"workload": f"identification_cube_{w.n_cells}", "n_cells": w.n_cells, "steps": steps,
            "ckpt_every": every, "forward_ms_per_step": 1e3 * t_plain / steps,
            "forward_record_ms_per_step": 1e3 * t_rec / steps, "adjoint_ms_per_step": 1e3 * t_adj / steps,
            "adjoint_forward_ratio": t_adj / t_plain, "grad_finite": bool(np.all(np.isfinite(gmu)))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="impact_bar_graded_8.1M")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the many-mesh batched-vs-sequential measurement")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the step on the once-refined workload")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the three-level cascade and shear-energy variant measurements")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward time measurement")
    ap.add_argument("--eager", action="store_true",
                    help="time the step launched eagerly instead of as a captured hipGraph")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the launch schedules of the headline workload first (the library's "
                         "defaults are the tuner's choice on it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the step has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        n = (1 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8}))
        return

    from paper_2104_02139_amd import hyperlag as H
    name = args.workload
    w = workloads()[name]()
    print(f"[bench] workload {name}: {w.n_cells} cells, {w.n_nodes} nodes", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    ctx = H.from_workload(w, device=0, stream=stream)
    ctx.compute_dt()
    schedules = None
    if args.autotune:
        t0 = time.perf_counter()
        schedules = {k: v[0] for k, v in ctx.autotune(reps=3).items()}
        print(f"[bench] autotune {time.perf_counter() - t0:.1f} s: {schedules}", file=sys.stderr, flush=True)

    if not args.eager:
        ctx.use_graph(True, 6)
    # warm-up (untimed; captures the graphs), also the MOOD statistics
    iters, p0 = [], []
    for _ in range(args.warmup):
        inf = ctx.step(0.0, info=True)
        iters.append(inf["mood_iters"])
        p0.append(inf["n_p0"])
    torch.cuda.synchronize()

    # timed region: K steps as submitted in production (captured hipGraph
    # unless --eager), no profiling events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.step(0.0, info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel launch times: K more steps with HIP events around every
    # launch (profiling runs the step eagerly)
    ctx.profile(True)
    ctx.profile_reset()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        ctx.step(0.0, info=False)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    kern = {k: ctx.profile_get(k) for k in PROFILED}
    ctx.profile(False)
    inf = ctx.step(0.0, info=True)
    iters.append(inf["mood_iters"])
    p0.append(inf["n_p0"])

    el = t1 - t0
    ms_per_step = 1e3 * el / args.steps
    value = w.n_cells * args.steps / el
    print(f"[bench] {ms_per_step:.3f} ms/step, {value:.4g} cell-updates/s", file=sys.stderr, flush=True)

    kb = kernel_bytes(w.dim, w.n_cells, w.n_nodes)
    total = {k: kern[k][0] * kern[k][1] for k in kern}
    dom = max(kb, key=lambda k: total.get(k, 0.0))
    avg_ms, launches = kern[dom]
    step_bytes = step_alg_bytes(w.dim, w.n_cells, w.n_nodes)
    # roofline of the dominant kernel on the algorithmic bytes of the step
    # it is part of (state in and out, constants, connectivity and node data
    # once), not on the intermediates the staged design adds
    achieved = step_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = read_traffic(dom, name)
    flop = read_valu(dom, name)
    stage_traffic = read_stage_traffic(name)
    step_flop = ALG_FLOP_PER_CELL[w.dim] * w.n_cells
    hbm_frac = (step_bytes / (HBM_PEAK_GBS * 1e9)) / (ms_per_step * 1e-3)
    fp64_frac = (step_flop / (FP64_PEAK_TFLOPS * 1e12)) / (ms_per_step * 1e-3)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "dim": w.dim, "n_cells": w.n_cells, "n_nodes": w.n_nodes,
                   "cascade": "P1->P0", "cfl": w.c_cfl, "launch": "eager" if args.eager else "hipGraph",
                   "numbering": "spatial (cells on a Hilbert curve, nodes by first use)"},
        "ms_per_step_profiled_eager": 1e3 * (t3 - t2) / args.steps,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": step_bytes,
                     "alg_bytes_per_cell": step_bytes / w.n_cells,
                     "avg_launch_ms": avg_ms, "launches": launches},
        # bytes each stage kernel moves as built (intermediates included)
        "kernel_design_bytes_per_launch": kb,
        # the same launch against the FP64 vector peak, from the committed
        # VALU counter summary (null when taken on another kernel source)
        "fp64_valu": None if flop is None or avg_ms <= 0 else {
            "kernel": dom, "achieved": flop / (avg_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": flop / (avg_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "flop_per_launch": flop},
        # alg_bytes: compulsory bytes of the whole step (state in and out,
        # constants, connectivity, node data, each once); measured: the
        # rocprofv3 HBM traffic of the four stage kernels (one launch each,
        # MOOD passes and the CFL reduction not included), null unless
        # taken on the current kernel source
        "step_roofline": {"alg_bytes_per_step": step_bytes, "alg_flop_per_step": step_flop,
                          "hbm_frac": hbm_frac, "fp64_frac": fp64_frac,
                          "classic_frac": max(hbm_frac, fp64_frac),
                          "measured_stage_bytes_per_step": None if stage_traffic is None
                          else sum(stage_traffic.values()),
                          "measured_hbm_frac": None if stage_traffic is None
                          else sum(stage_traffic.values()) / (HBM_PEAK_GBS * 1e9) / (ms_per_step * 1e-3)},
        "kernel_avg_ms": {k: kern[k][0] for k in kern},
        "kernel_launches": {k: kern[k][1] for k in kern},
        "mood": {"iters_mean": sum(iters) / len(iters), "first_order_frac_mean":
                 sum(p0) / len(p0) / w.n_cells},
        "adjoint_forward_ratio": None,
        "schedules": schedules,
        "kernel_source_sha1": kernel_source_hash(),
    }
    # what two plain kernels reach on this device (streaming copy, FP64
    # FMA), for reading the vendor-peak fractions above
    copy_gbs, fma_tf = H.measure_peaks(0, stream)
    out["device_peaks"] = {"copy_GBps": copy_gbs, "fp64_fma_TFLOPs": fma_tf,
                           "vendor_hbm_GBps": HBM_PEAK_GBS, "vendor_fp64_TFLOPs": FP64_PEAK_TFLOPS,
                           "roofline_achieved_over_copy": achieved / copy_gbs if copy_gbs > 0 else None}
    if not args.no_variants:
        print("[bench] scheme variants on the same workload", file=sys.stderr, flush=True)
        out["variants"] = [
            variant_measure(ctx, w, args.steps, args.warmup, not args.eager,
                            "cascade P1->P1+BJ->P0", cascade=3),
            variant_measure(ctx, w, args.steps, args.warmup, not args.eager,
                            "shear energy a=0", shear_a=0.0),
        ]
        if w.dim == 3 and name.startswith("impact_bar"):
            out["variants"] += [
                variant_measure(ctx, w, args.steps, args.warmup, not args.eager,
                                "boundary loads (far-end velocity, top traction)", setup=bar_loads(w)),
                variant_measure(ctx, w, args.steps, args.warmup, not args.eager,
                                "contact lid over the top face", setup=bar_lid(w)),
                variant_measure(ctx, jelly_material(w), args.steps, args.warmup, not args.eager,
                                "stiffened gas (droplet material, 3 m/s)", eos=1, sg_gamma=2.2, sg_pinf=1e6),
            ]
    if not args.no_variants and w.dim == 3 and name.startswith("impact_bar"):
        print("[bench] numbering, MOOD-heavy and configuration variants", file=sys.stderr, flush=True)
        ctx.close()
        del ctx
        out["variants"] += [
            workload_measure("shuffled input (random cell and node order, renumbered by the library)",
                             permuted(w, 1), args.steps, args.warmup, not args.eager),
            workload_measure("caller's numbering kept (generator order)", w, args.steps, args.warmup,
                             not args.eager, numbering=H.NUMBERING_KEEP),
        ]
        prep, frac = impact_noise(w, amp=1.0, xmax=0.4)
        v = workload_measure(f"MOOD-heavy: 1 m/s velocity noise on the impact region (x < 0.4, {frac:.3f} of the "
                             "cells), 10 steps timed from the first", w, 10, 0, not args.eager, prepare=prep)
        out["variants"].append(v)
        out["configs"] = [
            workload_measure("rotating cube 56^3 (1.05M tets)", workloads()["rotating_cube_1.05M"](),
                             args.steps, args.warmup, not args.eager),
            workload_measure("impact bar 240x60x60 (5.18M tets)", workloads()["impact_bar_5.2M"](),
                             args.steps, args.warmup, not args.eager),
        ]
    if not args.no_refined:
        print("[bench] the workload refined once on the GPU, stepped", file=sys.stderr, flush=True)
        out["refined_x8"] = refined_measure(w, args.steps, args.warmup, not args.eager)
    if not args.no_adjoint:
        print("[bench] adjoint vs forward on the identification cube", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_measure()
        out["adjoint_forward_ratio"] = out["adjoint"]["adjoint_forward_ratio"]
    if not args.no_batch:
        print("[bench] batched many-mesh step vs mesh-after-mesh launches", file=sys.stderr, flush=True)
        out["batch"] = batch_measure()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(name)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
