"""hl_measure_peaks: a streaming copy and independent FP64 FMAs reach a
plausible share of the vendor peaks (8 TB/s HBM, 78.6 TFLOP/s FP64
vector) and never exceed them; bad arguments are refused."""
import ctypes as C

import pytest

from paper_2104_02139_amd import hyperlag as H

pytestmark = pytest.mark.gpu


def test_peaks_are_plausible():
    gbs, tf = H.measure_peaks(0, None, 1 << 30)   # 2 GiB moved: past the 256 MB last-level cache
    print(f"[peaks] copy {gbs:.0f} GB/s, FP64 FMA {tf:.1f} TFLOP/s", flush=True)
    assert 1000.0 < gbs <= 8000.0 * 1.05
    assert 10.0 < tf <= 78.6 * 1.05


def test_bad_arguments_are_refused():
    L = H.load()
    a, b = C.c_double(), C.c_double()
    assert L.hl_measure_peaks(0, None, 1000, C.byref(a), C.byref(b)) == H.HL_E_INVALID
    assert L.hl_measure_peaks(0, None, (1 << 20) + 8, C.byref(a), C.byref(b)) == H.HL_E_INVALID
    assert L.hl_measure_peaks(0, None, 1 << 20, None, C.byref(b)) == H.HL_E_INVALID
