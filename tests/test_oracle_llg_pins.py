"""Pins of the oracle's full LLG time integration (eq. (9): precession and
damping, reduced time unit mu0|S|/(gamma J)).  Checked against closed forms
of a single spin in its anisotropy field (pure precession at alpha = 0;
damped spiral for alpha > 0), conservation of energy and spin length by the
precession, and the Lyapunov decrease of the energy with damping."""
import numpy as np

from paper_1804_07135_amd import inputs


def spin(theta, phi):
    s = np.zeros((3, 1, 1, 1))
    s[:, 0, 0, 0] = [np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)]
    return s


def angles(y):
    v = y[:, 0, 0, 0]
    return np.arccos(v[2] / np.linalg.norm(v)), np.arctan2(v[1], v[0])


def test_single_spin_precession(oracle):
    """alpha = 0: h = 2k s_z z, the spin precesses about z at 2 k cos(theta)
    with theta fixed."""
    k, th0, ph0, T = 0.4, 0.9, 0.3, 3.0
    r = oracle.llg_interval(spin(th0, ph0), 0.0, 0.0, k, 0.0, 0.0, T, 1e-11, 1e-11, 0.01)
    th, ph = angles(r["y"])
    assert abs(th - th0) < 1e-9
    expect = ph0 + 2 * k * np.cos(th0) * T
    assert abs(np.angle(np.exp(1j * (ph - expect)))) < 1e-9


def test_single_spin_damped_spiral(oracle):
    """alpha > 0: tan(theta) = tan(theta0) exp(-b t), b = 2 k alpha/(1+alpha^2),
    and phi = phi0 + (asinh(exp(b t)/tan(theta0)) - asinh(1/tan(theta0)))/alpha."""
    k, al, th0, ph0, T = 0.35, 0.2, 1.1, -0.4, 4.0
    b = 2 * k * al / (1 + al * al)
    c = np.tan(th0)
    r = oracle.llg_interval(spin(th0, ph0), 0.0, 0.0, k, 0.0, al, T, 1e-11, 1e-11, 0.01)
    th, ph = angles(r["y"])
    assert abs(th - np.arctan(c * np.exp(-b * T))) < 1e-9
    expect = ph0 + (np.arcsinh(np.exp(b * T) / c) - np.arcsinh(1 / c)) / al
    assert abs(np.angle(np.exp(1j * (ph - expect)))) < 1e-9


def test_precession_conserves_energy_and_length(oracle):
    """alpha = 0: dE/dt = -h . ds/dt = h . (s x h) = 0 and d|s|/dt = 0 (before
    the final renormalisation), so both hold up to the tolerance."""
    p = (1.0, 0.3, 0.1, 0.02)
    s = inputs.random_unit_spins((3, 1, 6, 7), seed=21)
    E0 = oracle.energy(s, *p)
    r = oracle.llg_interval(s, *p, 0.0, 1.5, 1e-10, 1e-10, 0.01)
    assert r["ok"]
    assert abs(oracle.energy(r["y"], *p) - E0) < 1e-7 * abs(E0)
    # the state moved (precession is not trivial)
    assert np.abs(r["y"] - s).max() > 1e-2


def test_damping_lowers_energy(oracle):
    """alpha > 0: dE/dt = -alpha/(1+alpha^2) |s x h|^2 <= 0."""
    p = (1.0, 0.3, 0.1, 0.02)
    s = inputs.random_unit_spins((3, 1, 6, 7), seed=22)
    E0 = oracle.energy(s, *p)
    f, h = oracle.llg_rhs(s, *p, 0.5)
    sxh = np.cross(s, h, axis=0)
    T = 1e-4
    r = oracle.llg_interval(s, *p, 0.5, T, 1e-12, 1e-12, T)
    dE = oracle.energy(r["y"], *p) - E0
    assert dE < 0
    assert abs(dE / (-0.5 / 1.25 * T * (sxh * sxh).sum()) - 1) < 1e-3


def test_rhs_parts(oracle):
    """The full right-hand side splits into precession and the damping term
    of the string method: f = -(s x h)/(1+a^2) + a/(1+a^2) f_damp."""
    p = (1.0, 0.25, 0.15, 0.03)
    s = inputs.random_unit_spins((3, 2, 4, 5), seed=23)
    al = 0.7
    f, h = oracle.llg_rhs(s, *p, al)
    fd, _ = oracle.rk_rhs(s, *p)
    expect = -np.cross(s, h, axis=0) / (1 + al * al) + al / (1 + al * al) * fd
    np.testing.assert_allclose(f, expect, atol=1e-13)
    assert np.abs((f * s).sum(0)).max() < 1e-13
