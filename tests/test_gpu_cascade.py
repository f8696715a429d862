"""Three-level MOOD cascade P1 -> P1 with the Barth-Jespersen limiter -> P0
(Section 3.5) through the C-ABI against the oracle: one step and CFL-run
parity with identical cascade levels, the many-mesh batch and the captured
graph equal to the eager single-mesh path bitwise, and the adjoint's refusal
of the limited cascade."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

from .parity_util import FIELDS, compare_states, fmt, max_err, pair

pytestmark = pytest.mark.gpu

ONE_STEP = 1e-12
HUNDRED = 1e-9

CASES = {
    "impact_bar_graded_16x4": lambda: W.impact_bar_3d(nx=16, ny=4, graded=True, seed=11),
    "impact_bar_24x6x6": lambda: W.impact_bar_3d(nx=24, ny=6, graded=False),
    "plane_wave_2d_n20": lambda: W.plane_wave_2d(n=20, amp=1e-3),
}


def _log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("case", list(CASES))
def test_one_step_parity_three_levels(case):
    """In the caller's numbering, so that the nodes sum their corners in
    the oracle's order: on the small 2D wave the nodal right-hand sides
    cancel to a few 1e-3 of their terms, and the limiter's ratios (M - W)
    / D of near-flat slopes carry that rounding, so another summation order
    moves v* by up to 5e-13 of its size (the spatial numbering is compared
    with the kept one in tests/test_gpu_numbering.py)."""
    w = CASES[case]()
    ctx, prob = pair(w, cascade=3, numbering=H.NUMBERING_KEEP)
    dt = prob.initial_dt()
    # a second step so that the state is no longer uniform
    info = ctx.step(dt)
    _, _, mk0, oi0 = prob.step(dt)
    assert np.array_equal(ctx.query("order"), mk0)
    dt = oi0.dt_next
    info = ctx.step(dt)
    s1, vs, mk, oi = prob.step(dt)
    e = compare_states(ctx, s1, vs)
    _log(f"[cascade3] {case}: errs {fmt(e)} levels gpu {np.bincount(ctx.query('order'), minlength=3)} "
         f"orc {np.bincount(mk, minlength=3)} mood {info['mood_iters']}/{oi.mood_iters}")
    assert np.array_equal(ctx.query("order"), mk)
    assert info["mood_iters"] == oi.mood_iters
    assert info["n_limited"] == oi.n_lim and info["n_p0"] == oi.n_p0
    assert max_err(e) <= ONE_STEP, fmt(e)


@pytest.mark.parametrize("case,steps", [("impact_bar_graded_16x4", 100), ("plane_wave_2d_n20", 100)])
def test_multi_step_parity_three_levels(case, steps):
    w = CASES[case]()
    ctx, prob = pair(w, cascade=3)
    ctx.compute_dt()
    dt = prob.initial_dt()
    flips = 0
    n_lim = 0
    for _ in range(steps):
        info = ctx.step(0.0)
        s1, vs, mk, oi = prob.step(dt)
        if not np.array_equal(ctx.query("order"), mk):
            flips += 1
        n_lim += oi.n_lim
        dt = oi.dt_next
    e = compare_states(ctx, prob.state)
    _log(f"[cascade3] {steps} steps {case}: {fmt(e)} mask-differing steps {flips}, limited cell-steps {n_lim}")
    assert n_lim > 0, "the case should use the limited level"
    assert flips == 0
    assert max_err(e) <= HUNDRED, fmt(e)


def test_batch_and_graph_equal_single_three_levels():
    ws = [W.impact_bar_3d(nx=16, ny=4, graded=True, seed=11), W.rotating_cube_3d(n=4, seed=2),
          W.impact_bar_3d(nx=10, ny=3, graded=False, seed=5)]
    prm = H.default_params(3, cascade=3)
    b = H.from_workloads(ws, params=prm)
    b.use_graph(True, 4)
    singles = [H.from_workload(w, params=prm) for w in ws]
    for _ in range(8):
        b.step_batch(None)
        for s in singles:
            s.step(0.0)
    st = b.state()
    no, co = b.node_offsets, b.cell_offsets
    order = b.query("order")
    for m, s in enumerate(singles):
        ss = s.state()
        for f in ("x", "vhat"):
            assert np.array_equal(st[f][no[m]:no[m + 1]], ss[f]), (m, f)
        for f in ("tau", "v", "e", "B"):
            assert np.array_equal(st[f][co[m]:co[m + 1]], ss[f]), (m, f)
        assert np.array_equal(order[co[m]:co[m + 1]], s.query("order"))
    assert (order == 1).any()


def test_adjoint_refuses_the_limited_cascade():
    w = W.rotating_cube_3d(n=2, seed=1)
    ctx = H.from_workload(w, params=H.default_params(3, cascade=3))
    with pytest.raises(H.HyperLagError):
        ctx.forward_record(2, 1)


def test_invalid_cascade_rejected():
    w = W.rotating_cube_3d(n=2, seed=1)
    ctx = H.from_workload(w)
    with pytest.raises(H.HyperLagError):
        ctx.set_params(H.default_params(3, cascade=4))
