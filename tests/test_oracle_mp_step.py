"""The FP64 oracle against a whole step evaluated in 50-digit arithmetic
(tests/mp_step.py, written separately from the paper and the readings;
it shares no code with the oracle).

On tiny meshes -- one Kuhn cube (6 tetrahedra), a 2 x 2 split square (8
triangles) with slip walls, a 12-tetrahedron bar hitting a slip wall --
both sides take the same seeded state through one step: the unlimited
candidate with detection off, and the full MOOD loop (eqs. PAD, RDMP;
Section 3.7).  The 50-digit values are exact far below FP64 roundoff, so
the oracle must agree to a few hundred ulps in every field, with
identical cascade choices, iteration counts and time steps.  A formula
slip on either side would show as an O(1) difference.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import workloads as W

from tests import mp_step as M

FIELDS = ("vhat", "tau", "v", "e", "B")
TOL = 1e-13    # normwise relative, per field
TOL_X = 1e-15  # positions (the displacement is tiny against x)


def _err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    num = np.abs(a - b).max()
    return num / den if den > 0 else num


def _perturbed(P, seed, scale):
    """A general smooth-ish state: tau, B and v perturbed cell by cell."""
    rng = np.random.default_rng(seed)
    st = P.state.copy()
    nc, d = P.mesh.nc, P.dim
    st.tau = st.tau * (1.0 + W.perturb_state(rng, nc, scale))
    for q in range(P.mesh.nB):
        st.B[:, q] += W.perturb_state(rng, nc, scale)
    st.v = st.v + W.perturb_state(rng, nc * d, scale * max(1.0, np.abs(st.v).max())).reshape(nc, d)
    k2 = 0.5 * np.sum(st.v * st.v, axis=1)
    st.e = k2 + 1e-3 * (1.0 + W.perturb_state(rng, nc, 0.1))
    return st


# (workload, perturbation (seed, scale) or None, oracle steps taken first)
CASES = {
    "kuhn_cube": (lambda: W.rotating_cube_3d(n=1, jitter=0.0), None, 0),
    "kuhn_cube_perturbed": (lambda: W.rotating_cube_3d(n=1, jitter=0.0), (1, 1e-3), 0),
    "split_square": (lambda: W.plane_wave_2d(n=2, amp=0.05), None, 0),
    "split_square_later": (lambda: W.plane_wave_2d(n=2, amp=0.05), None, 3),
    "split_square_perturbed": (lambda: W.plane_wave_2d(n=2, amp=0.05), (2, 1e-2), 0),
    "bar_on_wall": (lambda: W.impact_bar_3d(nx=2, ny=1, graded=False), None, 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("detect", [False, True])
def test_whole_step_matches_50_digit_evaluation(name, detect):
    make, pert, pre = CASES[name]
    w = make()
    P = O.Problem(w)
    dt = P.initial_dt()
    for _ in range(pre):
        _, _, _, info = P.step(dt)
        dt = info.dt_next
    st = P.state if pert is None else _perturbed(P, *pert)
    nc = P.mesh.nc
    if detect:
        s1, vs, mk, info = P.step(dt, state=st)
    else:
        s1, vs, mk, info = P.step(dt, state=st, mask=np.zeros(nc, np.uint8), replay=True)
    prm = dict(c_cfl=P.params.c_cfl, c_v=P.params.c_v, c_i=P.params.c_i, delta0=P.params.delta0,
               delta1=P.params.delta1, eps_tol=P.params.eps_tol)
    mpp = M.MPProblem(w.dim, w.x, w.cells, w.nwall, w.normals, w.rho0, w.mu, w.lam)
    sd = dict(x=st.x, vhat=st.vhat, tau=st.tau, v=st.v, e=st.e, B=st.B)
    new, vsm, mkm, im = mpp.step(sd, dt, prm, mask=None if detect else np.zeros(nc), detect=detect)
    out = mpp.pack(new)
    vsm = np.array([[float(p[i]) for i in range(w.dim)] for p in vsm])
    assert np.all(np.isfinite(vs)), "the case must keep the candidate finite"
    assert list(mk) == list(mkm)
    assert info.mood_iters == im["mood_iters"]
    assert info.n_flag_first == im["n_flag_first"]
    assert info.n_p0 == im["n_p0"]
    errs = {f: _err(getattr(s1, f), out[f]) for f in FIELDS}
    errs["vstar"] = _err(vs, vsm)
    assert max(errs.values()) <= TOL, errs
    assert _err(s1.x, out["x"]) <= TOL_X
    for k in ("dt_next", "dt_acoustic", "mass", "energy", "kinetic"):
        assert abs(info.as_dict()[k] - float(im[k])) <= TOL * abs(float(im[k])), k
    # the stored energy cancels (I1 - 3 ~ strain^2): its roundoff scale is
    # that of its terms, sum m (K + mu) / rho0
    scale = float(np.sum(P.m * (P.K + P.mu) / P.rho0))
    assert abs(info.elastic - float(im["elastic"])) <= TOL * scale
    mom = np.array(info.mom[:w.dim])
    ref = np.array([float(v) for v in im["mom"][:w.dim]])
    assert np.abs(mom - ref).max() <= TOL * max(np.abs(ref).max(), float(im["mass"]) * np.abs(st.v).max())
    if detect and name == "bar_on_wall":
        assert info.mood_iters >= 3   # the MOOD loop is exercised
