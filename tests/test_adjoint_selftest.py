"""Local derivatives of the adjoint step, on the host (no GPU): each
vector-Jacobian product in hl_adjoint.h (stress, impedance, chain-rule
div T, Crank-Nicolson and Euler B updates, simplex geometry, the corner
outer product C C^T/|C|, the nodal solve with 0..d wall directions) against
central differences of the forward function it differentiates, over random
inputs.  The same header is compiled into the GPU kernels."""
import ctypes as C
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2104_02139_amd", "libhl_selftest.so")

CASES = [("st_stress", ()), ("st_impedance", ()), ("st_divT3", ()), ("st_divT2", ()),
         ("st_cn3", ()), ("st_cn2", ()), ("st_euler3", ()), ("st_euler2", ()),
         ("st_geom3", ()), ("st_geom2", ()), ("st_outer3", ()), ("st_outer2", ()),
         ("st_node3", (3,)), ("st_node3", (2,)), ("st_node3", (1,)), ("st_node2", (2,)),
         ("st_node2", (1,))]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built; run `python -m paper_2104_02139_amd.build`")
    return C.CDLL(LIB)


@pytest.mark.parametrize("name,extra", CASES, ids=[f"{n}{e}" for n, e in CASES])
def test_local_vjp_matches_central_differences(lib, name, extra):
    f = getattr(lib, name)
    f.restype = C.c_double
    f.argtypes = [C.c_int] * (1 + len(extra))
    worst = f(200, *extra)
    # central differences with a relative step of 1e-6 (truncation ~1e-12,
    # roundoff ~1e-16 / 1e-6 per unit of conditioning): the mismatch is the
    # worst over 200 draws relative to the difference quotient, which some
    # draws make small.  Measured: <= 7.2e-7 (stress), <= 7e-8 elsewhere.
    # A wrong term, sign or index gives O(1).
    assert worst <= 5e-6, (name, extra, worst)
