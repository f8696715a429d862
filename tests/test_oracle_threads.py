"""The OpenMP build of the oracle (timed as the CPU baseline) gives
bitwise the serial build's results: every output cell and node is computed
by one thread in the serial order, sums over cells stay serial, and minima
and maxima do not depend on the order."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W


def _run(threads, w, steps, cascade):
    O.use_threads(threads)
    try:
        P = O.Problem(w, O.default_params(w.c_cfl, cascade=cascade))
        dt = P.initial_dt()
        infos, masks = [], []
        for _ in range(steps):
            _, vs, mk, info = P.step(dt)
            infos.append(info.as_dict())
            masks.append(mk.copy())
            dt = info.dt_next
        return P.state, vs, masks, infos
    finally:
        O.use_threads(False)


@pytest.mark.parametrize("make,cascade", [(lambda: W.impact_bar_3d(nx=16, ny=4, graded=True), 2),
                                          (lambda: W.plane_wave_2d(n=12, amp=0.05), 3)])
def test_threaded_oracle_is_bitwise_serial(make, cascade):
    w = make()
    a = _run(False, w, 5, cascade)
    b = _run(True, w, 5, cascade)
    for f in ("x", "vhat", "tau", "v", "e", "B"):
        assert np.array_equal(getattr(a[0], f), getattr(b[0], f)), f
    assert np.array_equal(a[1], b[1])
    for ma, mb in zip(a[2], b[2]):
        assert np.array_equal(ma, mb)
    assert a[3] == b[3]
    assert any(i["mood_iters"] > 1 for i in a[3])
