"""Launch schedules of the stage kernels: work items of `tile` consecutive
entities of one mesh (largest mesh first), walked by blocks of `block`
threads, optionally persistent (a few blocks per compute unit).  Every
entity is computed by one thread in a fixed order, so any schedule, and the
one the autotuner picks, must give bitwise the same steps as the default."""
import numpy as np
import pytest

from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import FIELDS

pytestmark = pytest.mark.gpu

SCHEDULES = [
    dict(tile=64, block=64, blocks_per_cu=1),      # persistent, few blocks
    dict(tile=512, block=128, blocks_per_cu=2),    # persistent, several items per block
    dict(tile=100, block=192, blocks_per_cu=0),    # ragged items, idle lanes
    dict(tile=1024, block=256, blocks_per_cu=8),
    dict(tile=8, block=64, blocks_per_cu=0),       # one pass of 8 nodes per block
]


def _run(ctx, steps, batch):
    masks = []
    for _ in range(steps):
        if batch:
            ctx.step_batch(None)
        else:
            ctx.step(0.0)
        masks.append(ctx.query("order").copy())
    return ctx.state(), masks


def _same(a, b):
    sa, ma = a
    sb, mb = b
    for f in FIELDS:
        assert np.array_equal(sa[f], sb[f]), f
    for x, y in zip(ma, mb):
        assert np.array_equal(x, y)


def _bar():
    # MOOD active: first-order cells appear within the first steps
    return W.impact_bar_3d(nx=16, ny=4, graded=True, seed=11)


def _family():
    ws = [W.rotating_cube_3d(n=3, seed=1), W.impact_bar_3d(nx=10, ny=3, graded=False, seed=2),
          W.rotating_cube_3d(n=5, seed=3), W.rotating_cube_3d(n=1, seed=4)]
    ws[2].mu = ws[2].mu * 1.7
    return ws


def _predict_default(cells_per_mesh, n_cu):
    """The predictor's default: T-cell items on T-thread blocks, T the
    largest of 256, 128, 64 that gives at least 8 items per CU."""
    for t in (256, 128):
        if sum(-(-n // t) for n in cells_per_mesh) >= 8 * n_cu:
            return dict(tile=t, block=t, blocks_per_cu=0)
    return dict(tile=64, block=64, blocks_per_cu=0)


def test_default_schedules():
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    w = _bar()
    ctx = H.from_workload(w)
    want = {"pack": dict(tile=256, block=256, blocks_per_cu=0),
            "node_agg": dict(tile=64, block=256, blocks_per_cu=0),
            "predict": _predict_default([w.n_cells], n_cu),
            "node_solve": dict(tile=32, block=256, blocks_per_cu=0),
            "update": dict(tile=256, block=256, blocks_per_cu=0)}
    for stage in H.STAGES:
        assert ctx.get_schedule(stage) == want[stage], stage
    assert want["predict"]["tile"] == 64   # 2400 cells: few items
    # a mesh with 8 items of 256 cells per CU takes 256-cell items
    big = W.rotating_cube_3d(n=48, seed=1)
    assert big.n_cells >= 8 * 256 * n_cu, (big.n_cells, n_cu)
    assert H.from_workload(big).get_schedule("predict") == dict(tile=256, block=256, blocks_per_cu=0)


@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
def test_schedule_does_not_change_results(sched):
    w = _bar()
    steps = 8
    ref = _run(H.from_workload(w), steps, False)
    assert sum(int(m.sum()) for m in ref[1]) > 0, "the case should exercise MOOD"
    ctx = H.from_workload(w)
    for stage in H.STAGES:
        ctx.set_schedule(stage, **SCHEDULES[sched])
        assert ctx.get_schedule(stage) == SCHEDULES[sched]
    print(f"[schedule] {SCHEDULES[sched]} on {w.n_cells} cells", flush=True)
    _same(ref, _run(ctx, steps, False))


def test_schedules_on_batch_with_graph():
    ws = _family()
    ref = _run(H.from_workloads(ws), 6, True)
    ctx = H.from_workloads(ws)
    for i, stage in enumerate(H.STAGES):
        ctx.set_schedule(stage, **SCHEDULES[i % len(SCHEDULES)])
    ctx.use_graph(True, 4)
    print(f"[schedule] batch of {len(ws)} meshes, graph, mixed schedules", flush=True)
    _same(ref, _run(ctx, 6, True))


def test_autotune_keeps_state_and_results():
    w = _bar()
    steps = 6
    ref = _run(H.from_workload(w), steps, False)
    ctx = H.from_workload(w)
    before = ctx.state()
    picked = ctx.autotune(reps=1)
    print(f"[autotune] {picked}", flush=True)
    after = ctx.state()
    for f in FIELDS:
        assert np.array_equal(before[f], after[f]), f
    for stage, (sch, ms) in picked.items():
        # node stages (8 lanes per node) may also take 1/8 or 1/4 of a block
        tiles = [m * sch["block"] for m in (1, 2, 4)]
        if stage in ("node_agg", "node_solve"):
            tiles += [sch["block"] // 8, sch["block"] // 4]
        assert sch["block"] in (64, 128, 256) and sch["tile"] in tiles, (stage, sch)
        assert ms > 0.0
    _same(ref, _run(ctx, steps, False))


def test_invalid_schedules_rejected():
    ctx = H.from_workload(W.rotating_cube_3d(n=2, seed=1))
    for bad in (dict(tile=0), dict(block=32), dict(block=320), dict(block=100),
                dict(blocks_per_cu=-1), dict(blocks_per_cu=65), dict(tile=(1 << 20) + 1)):
        with pytest.raises(H.HyperLagError):
            ctx.set_schedule("predict", **bad)
    with pytest.raises(ValueError):
        ctx.set_schedule("no_such_stage")


def _scattered(w, seed):
    """The workload's cells in a random order and held in that order
    (NUMBERING_KEEP): each 256-cell item then uses far more distinct nodes
    than a node tile of the one-item predictor holds (189 in 3D, 255 in 2D),
    so its items are cut until each part fits."""
    rng = np.random.default_rng(seed)
    pc = rng.permutation(w.n_cells)
    ctx = H.Context(0)
    ctx.set_numbering(H.NUMBERING_KEEP)
    cells = np.ascontiguousarray(w.cells[pc], dtype=np.int32)
    ctx.upload_mesh(w.dim, w.x, cells, w.nwall, w.normals)
    ctx.init_state(w.rho0[pc], w.mu[pc], w.lam[pc], w.v_cell[pc], w.v_node,
                   H.default_params(w.dim, c_cfl=w.c_cfl))
    return ctx, cells


@pytest.mark.parametrize("make", [lambda: W.impact_bar_3d(nx=16, ny=4, graded=True, seed=11),
                                  lambda: W.plane_wave_2d(n=24, amp=0.05, seed=2)])
def test_predict_items_cut_to_fit_node_tiles(make):
    w = make()
    tiled, cells = _scattered(w, 5)
    first = len(np.unique(cells[:256]))
    assert first > (189 if w.dim == 3 else 255), first
    plain, _ = _scattered(w, 5)
    # the persistent predictor walks its items with no node tiles
    plain.set_schedule("predict", tile=512, block=128, blocks_per_cu=2)
    tiled.set_schedule("predict", tile=256, block=256)
    print(f"[schedule] node tiles on a scattered {w.dim}D mesh of {w.n_cells} cells "
          f"({first} nodes in the first 256 cells)", flush=True)
    _same(_run(plain, 8, False), _run(tiled, 8, False))
