"""The allocation-free acoustic time step (hl_acoustic_dt_noalloc) against
the context's hl_compute_dt, bitwise, on two calls in a row (the second
with a smaller mesh), through the C-ABI, with the state in caller-owned
device memory and the call enqueued on a torch stream."""
import numpy as np
import pytest

from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0").to(dtype).contiguous()


def _noalloc(st, w, c_cfl):
    import torch
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    H.acoustic_dt_noalloc(_dev(st["x"], torch.float64), _dev(w.cells, torch.int32), _dev(w.rho0, torch.float64),
                          _dev(w.mu, torch.float64), _dev(w.lam, torch.float64), _dev(st["tau"], torch.float64),
                          c_cfl, out, device=0, stream=stream)
    torch.cuda.current_stream().synchronize()
    return float(out.item())


def test_noalloc_dt_equals_compute_dt_twice():
    import torch
    torch.cuda.set_device(0)
    for w, steps in ((W.impact_bar_3d(nx=24, ny=6, graded=False), 4), (W.plane_wave_2d(n=7, amp=0.05), 2)):
        ctx = H.from_workload(w, stream=torch.cuda.current_stream())
        ctx.compute_dt()
        for _ in range(steps):
            ctx.step(0.0, info=False)
        ref = ctx.compute_dt()          # acoustic bound of the current state
        got = _noalloc(ctx.state(), w, w.c_cfl)
        assert got == ref, (got, ref)


def test_noalloc_rejects_bad_arguments():
    import torch
    w = W.rotating_cube_3d(n=2)
    st = {"x": w.x, "tau": 1.0 / w.rho0}
    bad_cells = w.cells.copy()
    bad_cells[3, 2] = w.n_nodes + 5
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    H.acoustic_dt_noalloc(_dev(w.x, torch.float64), _dev(bad_cells, torch.int32), _dev(w.rho0, torch.float64),
                          _dev(w.mu, torch.float64), _dev(w.lam, torch.float64), _dev(st["tau"], torch.float64),
                          0.25, out)
    torch.cuda.synchronize()
    assert np.isnan(float(out.item()))
    with pytest.raises(H.HyperLagError):
        H.acoustic_dt_noalloc(_dev(w.x, torch.float64), _dev(w.cells, torch.int32), _dev(w.rho0, torch.float64),
                              _dev(w.mu, torch.float64), _dev(w.lam, torch.float64), _dev(st["tau"], torch.float64),
                              -1.0, out)
