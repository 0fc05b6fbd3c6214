"""Pins of the FW-H oracle (oracle/fwh.py) against what the paper and the mathematics fix.

* Stationary monopole and dipole in a uniform stream, the paper's verification cases
  (Appendix C): sphere of radius 1 with 30 equal-area polar bands x 45 azimuthal panels,
  dt / T = 0.02, observers at 20 (monopole) and 100 (dipole) from the source, the
  paper's Mach vectors.  The exact pressure follows from the closed-form potential.
  The bars are what the discretisation allows: the surface quadrature and the time
  interpolation are second and fourth order; measured errors are 4e-5 .. 6e-4
  (monopole) and 7e-4 .. 4e-3 (dipole), relative RMS.
* Convergence: halving the panel size cuts the error by about four (for a weak
  source: the sampled source strengths carry quadratic terms that the linear closed
  form lacks, an error floor near 1e-3 at unit amplitude).
* Quiescent samples (rho0, no disturbance velocity, p0) radiate exactly nothing.
* Spanwise copies: the sum over copies shifted by s_k at observer x equals the sum of
  single-copy results at observers x - s_k (translation invariance; holds to round-off).
"""
import numpy as np
import pytest

from oracle import fwh
from paper_2501_05709_amd import workloads as W

CASES = [("monopole", (0.0, 0.0, 0.0), 20.0, 2e-4), ("monopole", (0.0, 0.0, 0.5), 20.0, 5e-4),
         ("monopole", (0.5, 0.1, 0.5), 20.0, 1e-3), ("monopole", (0.7, 0.1, 0.5), 20.0, 2e-3),
         ("dipole", (0.0, 0.0, 0.4), 100.0, 4e-3), ("dipole", (0.4, 0.0, 0.4), 100.0, 4e-3),
         ("dipole", (0.6, 0.0, 0.4), 100.0, 5e-3), ("dipole", (0.8, 0.0, 0.4), 100.0, 1e-2)]


def observer(dist, polar, azimuth=0.7):
    return dist * np.array([np.sin(polar) * np.cos(azimuth), np.sin(polar) * np.sin(azimuth), np.cos(polar)])


def run(c, x, **kw):
    return fwh.observer_pressure(c["points"], c["normals"], c["areas"], c["rho"], c["u"], c["p"], c["dt"], x,
                                 c["mach"], c["c0"], c["rho0"], c["p0"], **kw)


def exact(c, x, t):
    return W.stationary_source(c["kind"], x[None], t, c["mach"], c["c0"], c["rho0"], amplitude=c["amplitude"],
                               omega=c["omega"])[2][:, 0]


def rms_err(p, ref):
    return np.sqrt(np.mean((p - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))


@pytest.mark.parametrize("kind,mach,dist,tol", CASES)
def test_stationary_source_matches_closed_form(kind, mach, dist, tol):
    c = W.acoustic_case(kind, mach)
    for polar in (0.3, 1.2, 2.5):
        x = observer(dist, polar)
        t, p, pT, pL = run(c, x)
        assert t.size > 500
        err = rms_err(p, exact(c, x, t))
        assert err <= tol, (polar, err)
        assert np.allclose(p, pT + pL, rtol=0, atol=1e-14 * np.abs(p).max())


def test_error_falls_with_panel_size():
    # a weak source: the samples carry the quadratic terms of the source strengths,
    # which the linear closed form lacks; at unit amplitude they set a floor near 1e-3
    errs = []
    for n_polar, n_az in ((15, 23), (30, 45), (60, 90)):
        c = W.acoustic_case("dipole", (0.4, 0.0, 0.4), n_polar=n_polar, n_azimuth=n_az, periods=4,
                            amplitude=0.01)
        x = observer(100.0, 0.3)
        t, p, _, _ = run(c, x)
        errs.append(rms_err(p, exact(c, x, t)))
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0, errs


def test_quiescent_samples_radiate_nothing():
    c = W.acoustic_case("monopole", (0.3, 0.0, 0.2), periods=3)
    rho = np.full_like(c["rho"], c["rho0"])
    p = np.full_like(c["p"], c["p0"])
    u = np.zeros_like(c["u"])
    _, pp, _, _ = fwh.observer_pressure(c["points"], c["normals"], c["areas"], rho, u, p, c["dt"],
                                        observer(20.0, 1.0), c["mach"], c["c0"], c["rho0"], c["p0"])
    assert np.abs(pp).max() == 0.0


def test_spanwise_copies_equal_shifted_observers():
    c = W.acoustic_case("monopole", (0.2, 0.0, 0.0), periods=6, n_polar=10, n_azimuth=15)
    x = observer(20.0, 1.1)
    shift = np.array([0.0, 0.0, 2.5])
    n = 5
    t, p, _, _ = run(c, x, n_copies=n, shift=shift)
    total = np.zeros_like(p)
    for s in fwh.copy_shifts(n, shift):
        total += run(c, x - s, t_grid=t)[1]
    assert np.abs(p - total).max() <= 1e-12 * np.abs(p).max()
