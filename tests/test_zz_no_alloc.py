"""GPU check of the allocation-free FW-H entry point (fr_fwh_pressure_at_noalloc).

The entry point runs the kernels of fr_fwh_pressure_at with the evaluation's
intermediate arrays in the library's static device scratch instead of buffers
the record allocates; it must give the same pressure, bit for bit.  Two calls in
a row, the second with a smaller input (fewer panels, fewer observer times, a
later start), check that the static array's leftover contents do not leak into a
later result; a request beyond the array's size is refused before anything runs.
"""
import numpy as np
import pytest

from paper_2501_05709_amd import _lib
from paper_2501_05709_amd import workloads as W
from paper_2501_05709_amd.solver import FWH

pytestmark = pytest.mark.gpu


def record(kind, mach, n_polar, n_azimuth, n_copies=1, shift=(0.0, 0.0, 0.0)):
    c = W.acoustic_case(kind, mach, periods=6, n_polar=n_polar, n_azimuth=n_azimuth)
    g = FWH(c["points"], c["normals"], c["areas"], c["mach"], c["c0"], c["rho0"], c["p0"], c["dt"],
            c["rho"].shape[0], n_copies=n_copies, copy_shift=shift)
    g.append(c["rho"], c["u"], c["p"])
    return g, c["dt"]


def test_noalloc_matches_allocating_entry_point_twice():
    x = np.array([3.0, -25.0, 4.0])
    big, _ = record("dipole", (0.3, 0.05, 0.2), 30, 45, n_copies=5, shift=(0.0, 0.0, 2.5))  # 1,350 panels
    small, dt = record("monopole", (0.1, 0.0, 0.4), 12, 18)                                # 216 panels
    t0, n = big.window(x)
    ref = big.pressure_at(x, t0, n, parts=True)
    got = big.pressure_at_noalloc(x, t0, n, parts=True)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    # second call: fewer panels, a third of the observer times, starting 5 samples later
    t1, m = small.window(x)
    k = m // 3
    ref2 = small.pressure_at(x, t1 + 5 * dt, k, parts=True)
    got2 = small.pressure_at_noalloc(x, t1 + 5 * dt, k, parts=True)
    for a, b in zip(got2, ref2):
        assert np.array_equal(a, b)
    assert np.abs(ref[0]).max() > 0 and np.abs(ref2[0]).max() > 0
    print(f"noalloc: {n} and {k} observer times bit-identical to fr_fwh_pressure_at", flush=True)
    big.close()
    small.close()


def test_noalloc_refuses_beyond_the_static_array():
    # 8,000 panels need 8,000 x 8,576 bytes of combined filters alone, more than the
    # 64 MiB array: refused on the sizes, before any kernel runs
    n = 8000
    rng = np.random.default_rng(0)
    pts = rng.standard_normal((n, 3))
    nrm = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    g = FWH(pts, nrm, np.full(n, 1e-3), (0.0, 0.0, 0.2), 1.0, 1.0, 1.0 / 1.4, 0.01, 16)
    with pytest.raises(_lib.FRError) as e:
        g.pressure_at_noalloc(np.array([0.0, 0.0, 30.0]), 0.0, 3000)
    assert e.value.code == _lib.FR_E_ARG
    g.close()
