"""The printed set-up of the paper's worked cases (tests/golden/paper_setup.txt) against
the generators and constants that use it, and the exact source field of the FW-H
verification cases against what mathematics fixes.

* The verification set-up of Appendix C (source, medium, data surface, time step, observer
  distances, Mach vectors, RMS window) is what the generator and the oracle's pins use.
* The objective's penalty constants (Section 3.4) are the library's.
* In a medium at rest the exact field reduces to the textbook spherical waves: a monopole
  p' = rho0 omega A / (4 pi r) sin(omega (t - r / c0)), and its x2 derivative for the dipole.
* In a moving medium (the paper's Mach vectors) the field solves the linear convected
  equations: rho0 D u / Dt + grad p' = 0 and D rho' / Dt + rho0 div u = 0, D = d/dt + c0 M.grad,
  checked by central differences.
"""
import importlib.util
import inspect
import pathlib

import numpy as np
import pytest

from paper_2501_05709_amd import mads
from paper_2501_05709_amd import workloads as W

HERE = pathlib.Path(__file__).parent


def setup():
    out = {}
    for line in (HERE / "golden" / "paper_setup.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        key, rest = line.split("=", 1)
        value, cite = rest.split("|", 1)
        assert cite.strip(), key
        vecs = [[float(x) for x in v.split(",")] for v in value.split(";")]
        out[key.strip()] = vecs if len(vecs) > 1 else (vecs[0][0] if len(vecs[0]) == 1 else vecs[0])
    return out


G = setup()


def test_generator_defaults_are_the_printed_verification_setup():
    d = {k: v.default for k, v in inspect.signature(W.acoustic_case).parameters.items()}
    assert d["amplitude"] == G["amplitude"]
    assert d["omega"] == G["omega_over_pi"] * np.pi
    assert d["c0"] == G["c0"] and d["rho0"] == G["rho0"] and d["gamma"] == G["gamma"]
    assert d["radius"] == G["radius"] and d["n_polar"] == G["n_polar"] and d["n_azimuth"] == G["n_azimuth"]
    assert d["dt_over_T"] == G["dt_over_T"]
    c = W.acoustic_case("monopole", (0.0, 0.0, 0.0), periods=1)
    # ideal gas: p0 = rho0 c0^2 / gamma (Appendix C)
    assert np.isclose(c["p0"], G["rho0"] * G["c0"] ** 2 / G["gamma"], rtol=1e-15)
    assert np.isclose(c["dt"], G["dt_over_T"] * 2.0 / G["omega_over_pi"], rtol=1e-15)
    # equal-area panels over the whole sphere, 30 x 45 of them
    assert c["areas"].size == G["n_polar"] * G["n_azimuth"]
    assert np.allclose(c["areas"], c["areas"][0], rtol=1e-12)
    assert np.isclose(c["areas"].sum(), 4.0 * np.pi * G["radius"] ** 2, rtol=1e-12)
    assert np.allclose(np.linalg.norm(c["points"], axis=1), G["radius"], rtol=1e-12)


def test_oracle_pins_run_the_printed_cases():
    spec = importlib.util.spec_from_file_location("fwh_pins", HERE / "test_oracle_fwh.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mono = [list(m) for k, m, dist, _ in mod.CASES if k == "monopole"]
    dip = [list(m) for k, m, dist, _ in mod.CASES if k == "dipole"]
    assert mono == G["monopole_mach"] and dip == G["dipole_mach"]
    assert {dist for k, _, dist, _ in mod.CASES if k == "monopole"} == {G["monopole_distance"]}
    assert {dist for k, _, dist, _ in mod.CASES if k == "dipole"} == {G["dipole_distance"]}
    # the record those pins judge covers the printed RMS window
    assert inspect.signature(W.acoustic_case).parameters["periods"].default >= G["rms_periods"] + 1
    assert int(G["rms_periods"] / G["dt_over_T"]) == 500  # the pins' minimum record length
    assert "t.size > 500" in inspect.getsource(mod.test_stationary_source_matches_closed_form)


def test_objective_constants_are_the_printed_ones():
    assert (mads.EPS_LIFT, mads.EPS_DRAG) == (G["eps_lift"], G["eps_drag"])


def _points(rng, n, rmin, rmax):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return d * rng.uniform(rmin, rmax, size=(n, 1))


def test_field_at_rest_is_the_textbook_spherical_wave():
    A, w, c0, rho0 = G["amplitude"], G["omega_over_pi"] * np.pi, G["c0"], G["rho0"]
    k = w / c0
    rng = np.random.default_rng(3)
    x = _points(rng, 40, 0.5, 120.0)
    t = np.linspace(0.0, 0.4, 23)
    r = np.linalg.norm(x, axis=1)
    th = w * (t[:, None] - r[None] / c0)
    rho_p, u, p = W.stationary_source("monopole", x, t, (0.0, 0.0, 0.0), c0, rho0, amplitude=A, omega=w)
    p_ref = rho0 * w * A / (4 * np.pi * r) * np.sin(th)
    u_ref = A / (4 * np.pi) * (x / r[:, None])[None] * ((k / r) * np.sin(th) - np.cos(th) / r ** 2)[:, :, None]
    assert np.allclose(p, p_ref, rtol=0, atol=1e-13 * np.abs(p_ref).max())
    assert np.allclose(u, u_ref, rtol=0, atol=1e-13 * np.abs(u_ref).max())
    assert np.allclose(rho_p, p_ref / c0 ** 2, rtol=0, atol=1e-13 * np.abs(p_ref).max() / c0 ** 2)
    ax = int(G["dipole_axis"]) - 1
    rho_p, u, p = W.stationary_source("dipole", x, t, (0.0, 0.0, 0.0), c0, rho0, amplitude=A, omega=w, axis=ax)
    p_ref = -rho0 * w * A / (4 * np.pi) * (x[:, ax] / r)[None] * ((k / r) * np.cos(th) + np.sin(th) / r ** 2)
    assert np.allclose(p, p_ref, rtol=0, atol=1e-13 * np.abs(p_ref).max())
    # amplitude on the axis at the printed distance
    R = G["dipole_distance"]
    amp = rho0 * w * A / (4 * np.pi) * np.sqrt(k ** 2 / R ** 2 + 1 / R ** 4)
    xa = np.zeros((1, 3))
    xa[0, ax] = R
    ta = np.linspace(0.0, 2 * np.pi / w, 2001)
    pa = W.stationary_source("dipole", xa, ta, (0.0, 0.0, 0.0), c0, rho0, amplitude=A, omega=w, axis=ax)[2]
    assert np.isclose(np.abs(pa).max(), amp, rtol=1e-5)


@pytest.mark.parametrize("kind,mach", [("monopole", m) for m in G["monopole_mach"]] +
                         [("dipole", m) for m in G["dipole_mach"]])
def test_field_solves_the_convected_acoustic_equations(kind, mach):
    A, w, c0, rho0 = G["amplitude"], G["omega_over_pi"] * np.pi, G["c0"], G["rho0"]
    M = np.asarray(mach)
    ax = int(G["dipole_axis"]) - 1
    rng = np.random.default_rng(7)
    x = _points(rng, 12, 3.0, 30.0)
    t0 = np.array([0.013, 0.071])
    res = _convected_residuals(kind, M, M, x, t0, A, w, c0, rho0, ax)
    assert max(res) <= 1e-5, res
    # a planted mistake is seen: the field of the opposite stream fails the same equations
    if np.any(M):
        assert max(_convected_residuals(kind, -M, M, x, t0, A, w, c0, rho0, ax)) > 1e-2


def _convected_residuals(kind, M_field, M, x, t0, A, w, c0, rho0, ax, hx=1e-3, ht=2e-6):
    """Relative residuals of the momentum and continuity equations of a stream of Mach
    vector M, for the exact field of a source in a stream of Mach vector M_field."""

    def f(xx, tt):
        return W.stationary_source(kind, xx, tt, M_field, c0, rho0, amplitude=A, omega=w, axis=ax)

    dt = [(a - b) / (2 * ht) for a, b in zip(f(x, t0 + ht), f(x, t0 - ht))]
    dx = []
    for i in range(3):
        e = np.zeros(3)
        e[i] = hx
        dx.append([(a - b) / (2 * hx) for a, b in zip(f(x + e, t0), f(x - e, t0))])
    # D/Dt = d/dt + c0 M.grad
    Drho = dt[0] + c0 * sum(M[i] * dx[i][0] for i in range(3))
    Du = dt[1] + c0 * sum(M[i] * dx[i][1] for i in range(3))
    gradp = np.stack([dx[i][2] for i in range(3)], axis=-1)
    divu = sum(dx[i][1][..., i] for i in range(3))
    mom = rho0 * Du + gradp
    cont = Drho + rho0 * divu
    scale_m = np.abs(rho0 * dt[1]).max() + np.abs(gradp).max()
    scale_c = np.abs(dt[0]).max() + np.abs(rho0 * divu).max()
    return np.abs(mom).max() / scale_m, np.abs(cont).max() / scale_c
