"""GPU parity of the far-field acoustic step (fr_fwh_*) against the FW-H oracle.

Bar: FP64 throughout, so the acoustic pressure and its thickness and loading parts
agree with the oracle to 1e-12 of their largest magnitude, on the same observer-time
grid (start within 1e-12 relative, same length).  Index work (the window) is exact.
Cases: the paper's stationary monopole and dipole verification set-ups in streams of
several Mach vectors, spanwise copies, records appended in pieces, the error paths,
and, at the benchmark's full size, the copy/observer translation identity.
"""
import numpy as np
import pytest

from oracle import fwh
from paper_2501_05709_amd import _lib
from paper_2501_05709_amd import workloads as W
from paper_2501_05709_amd.solver import FWH

pytestmark = pytest.mark.gpu


def make(c, n_copies=1, shift=(0.0, 0.0, 0.0), capacity=None):
    nt = c["rho"].shape[0]
    return FWH(c["points"], c["normals"], c["areas"], c["mach"], c["c0"], c["rho0"], c["p0"], c["dt"],
               capacity or nt, n_copies=n_copies, copy_shift=shift)


def observer(dist, polar, azimuth=0.7):
    return dist * np.array([np.sin(polar) * np.cos(azimuth), np.sin(polar) * np.sin(azimuth), np.cos(polar)])


def close(a, b, tol=1e-12):
    return np.abs(a - b).max() <= tol * np.abs(b).max()


@pytest.mark.parametrize("kind,mach,dist", [("monopole", (0.0, 0.0, 0.0), 20.0), ("monopole", (0.7, 0.1, 0.5), 20.0),
                                            ("dipole", (0.0, 0.0, 0.4), 100.0), ("dipole", (0.8, 0.0, 0.4), 100.0)])
def test_pressure_matches_oracle(kind, mach, dist):
    c = W.acoustic_case(kind, mach, periods=6)
    g = make(c)
    g.append(c["rho"], c["u"], c["p"])
    for polar in (0.3, 2.5):
        x = observer(dist, polar)
        t, p, pT, pL = g.pressure(x, parts=True)
        to, po, pTo, pLo = fwh.observer_pressure(c["points"], c["normals"], c["areas"], c["rho"], c["u"], c["p"],
                                                 c["dt"], x, c["mach"], c["c0"], c["rho0"], c["p0"])
        assert t.size == to.size
        assert abs(t[0] - to[0]) <= 1e-12 * abs(to[0])
        assert close(p, po) and close(pT, pTo) and close(pL, pLo)
        print(f"{kind} {mach} polar {polar}: max |p - p_oracle| / max |p| = "
              f"{np.abs(p - po).max() / np.abs(po).max():.2e}", flush=True)


def test_copies_match_oracle():
    c = W.acoustic_case("monopole", (0.2, 0.05, 0.0), periods=8, n_polar=12, n_azimuth=18)
    shift = (0.0, 0.0, 3.0)
    g = make(c, n_copies=7, shift=shift)
    g.append(c["rho"], c["u"], c["p"])
    x = observer(25.0, 1.0)
    t, p = g.pressure(x)
    to, po, _, _ = fwh.observer_pressure(c["points"], c["normals"], c["areas"], c["rho"], c["u"], c["p"], c["dt"], x,
                                         c["mach"], c["c0"], c["rho0"], c["p0"], n_copies=7, shift=shift)
    assert t.size == to.size and close(p, po)


def test_pieces_equal_whole_and_errors():
    c = W.acoustic_case("dipole", (0.3, 0.0, 0.3), periods=4, n_polar=10, n_azimuth=16)
    nt = c["rho"].shape[0]
    a, b = make(c), make(c)
    a.append(c["rho"], c["u"], c["p"])
    for k in range(0, nt, 37):
        b.append(c["rho"][k:k + 37], c["u"][k:k + 37], c["p"][k:k + 37])
    assert a.samples() == b.samples() == nt
    x = observer(100.0, 0.8)
    assert np.array_equal(a.pressure(x)[1], b.pressure(x)[1])
    with pytest.raises(_lib.FRError) as e:
        b.append(c["rho"][:1], c["u"][:1], c["p"][:1])
    assert e.value.code == _lib.FR_E_ARG
    short = make(c)
    short.append(c["rho"][:6], c["u"][:6], c["p"][:6])
    with pytest.raises(_lib.FRError) as e:
        short.pressure(x)
    assert e.value.code == _lib.FR_E_STATE
    with pytest.raises(_lib.FRError) as e:
        FWH(c["points"], c["normals"], c["areas"], (0.8, 0.0, 0.7), c["c0"], c["rho0"], c["p0"], c["dt"], 16)
    assert e.value.code == _lib.FR_E_ARG


@pytest.mark.timeout(600)
def test_full_size_copies_equal_shifted_observers():
    """The benchmark's data surface (24,000 panels, 4,332 samples, 125 spanwise copies):
    the sum over copies at observer x equals the sum of single-copy results at x - s_k,
    on the copies' observer grid (translation invariance, any size; FP64 sums in a
    different order, so to 1e-12 of the largest magnitude)."""
    case = W.fwh_airfoil_case(seed=0)
    n = case["n_copies"]
    args = (case["points"], case["normals"], case["areas"], case["mach"], case["c0"], case["rho0"], case["p0"],
            case["dt"], case["n_samples"])
    g = FWH(*args, n_copies=n, copy_shift=case["copy_shift"])
    one = FWH(*args)
    for rho, u, p in W.fwh_airfoil_samples(case):
        g.append(rho, u, p)
        one.append(rho, u, p)
    x = case["observer"]
    t, p = g.pressure(x)
    print(f"full surface: {case['points'].shape[0]} panels x {n} copies, {t.size} observer times, "
          f"{g.time_ms():.1f} ms", flush=True)
    total = np.zeros_like(p)
    for s in fwh.copy_shifts(n, case["copy_shift"]):
        total += one.pressure_at(x - s, t[0], t.size)
    assert np.isfinite(p).all() and np.abs(p).max() > 0
    assert close(p, total)


def test_copies_beyond_the_combined_filter_match_oracle():
    """Copies whose arrival delays spread over more than 256 samples are summed copy by
    copy; nearer ones through one combined filter per panel.  Both against the oracle:
    a monopole sphere with 5 copies 200 apart heard from 20 away (spread about 280
    samples), and with 5 copies 2.5 apart (spread of a few samples)."""
    c = W.acoustic_case("monopole", (0.2, 0.0, 0.0), periods=9, n_polar=8, n_azimuth=12)
    x = np.array([20.0, 3.0, 1.0])
    for shift in (np.array([0.0, 0.0, 200.0]), np.array([0.0, 0.0, 2.5])):
        g = FWH(c["points"], c["normals"], c["areas"], c["mach"], c["c0"], c["rho0"], c["p0"], c["dt"],
                c["rho"].shape[0], n_copies=5, copy_shift=shift)
        g.append(c["rho"], c["u"], c["p"])
        t, p = g.pressure(x)
        to, po, _, _ = fwh.observer_pressure(c["points"], c["normals"], c["areas"], c["rho"], c["u"], c["p"],
                                             c["dt"], x, c["mach"], c["c0"], c["rho0"], c["p0"], n_copies=5,
                                             shift=shift)
        spread = np.ptp(fwh.radii(x[None], (c["points"][None] + fwh.copy_shifts(5, shift)[:, None]).reshape(-1, 3),
                                  c["mach"])[1]) / c["c0"] / c["dt"]
        print(f"copies {shift[2]:g} apart: delay spread {spread:.0f} samples, {t.size} observer times", flush=True)
        assert t.size == to.size and t.size > 10
        assert close(p, po)


def test_panels_of_both_summation_paths_in_one_chunk_match_oracle():
    """Panels that need the copy-by-copy path and panels that take the combined filter,
    interleaved so that every chunk of the summation holds both: a monopole sphere 20 from
    the observer (5 copies 200 apart: delays spread about 285 samples) and the same samples
    on a sphere moved 80 further away (spread about 233 samples).  Against the oracle."""
    c = W.acoustic_case("monopole", (0.2, 0.0, 0.0), periods=12, n_polar=7, n_azimuth=11)
    x = np.array([20.0, 3.0, 1.0])
    shift = np.array([0.0, 0.0, 200.0])
    n = c["points"].shape[0]
    order = np.ravel(np.column_stack([np.arange(n), n + np.arange(n)]))   # A0, B0, A1, B1, ...
    pts = np.concatenate([c["points"], c["points"] + np.array([-80.0, 0.0, 0.0])])[order]
    nrm = np.concatenate([c["normals"], c["normals"]])[order]
    area = np.concatenate([c["areas"], c["areas"]])[order]
    rho = np.concatenate([c["rho"], c["rho"]], axis=1)[:, order]
    u = np.concatenate([c["u"], c["u"]], axis=1)[:, order]
    p = np.concatenate([c["p"], c["p"]], axis=1)[:, order]
    R = fwh.radii(x[None], (pts[None] + fwh.copy_shifts(5, shift)[:, None]).reshape(-1, 3), c["mach"])[1]
    spread = np.ptp(R.reshape(5, -1), axis=0) / c["c0"] / c["dt"]
    assert spread[0::2].min() > 256 >= spread[1::2].max()   # both paths present, alternating
    g = FWH(pts, nrm, area, c["mach"], c["c0"], c["rho0"], c["p0"], c["dt"], rho.shape[0], n_copies=5,
            copy_shift=shift)
    g.append(rho, u, p)
    t, pr = g.pressure(x)
    to, po, _, _ = fwh.observer_pressure(pts, nrm, area, rho, u, p, c["dt"], x, c["mach"], c["c0"], c["rho0"],
                                         c["p0"], n_copies=5, shift=shift)
    print(f"{len(pts)} panels, spreads {spread[1::2].max():.0f} and {spread[0::2].min():.0f} samples, "
          f"{t.size} observer times", flush=True)
    assert t.size == to.size and t.size > 100
    assert close(pr, po)
