"""Pins of the oracle's adaptive Runge-Kutta step 1 (Sec. III: each image is
evolved over an interval by explicit embedded RK with adaptive step size;
damping term of eq. (9), Appendix).  Checked against what the mathematics
fixes, not against the integrator's own formulas: the Runge-Kutta order
conditions of the Dormand-Prince pair, the closed-form damped rotation of a
single spin in its anisotropy field, the convergence order of fixed steps,
the scaling of the embedded error estimate, the Lyapunov property of the
damping flow and stationarity of an exact minimum."""
import numpy as np
import pytest

from paper_1804_07135_amd import inputs


def single_spin(theta):
    s = np.zeros((3, 1, 1, 1))
    s[0, 0, 0, 0] = np.sin(theta)
    s[2, 0, 0, 0] = np.cos(theta)
    return s


def exact_theta(theta0, k, t):
    # one spin, energy -k s_z^2, field 2k s_z z: damping flow gives
    # d theta/dt = -k sin(2 theta), i.e. tan(theta) = tan(theta0) exp(-2 k t)
    return np.arctan(np.tan(theta0) * np.exp(-2.0 * k * t))


def test_tableau_order_conditions(oracle):
    """Butcher order conditions: order 5 for b (the propagated solution),
    order 4 for b* (the embedded one), and the row-sum condition."""
    a, b, bs, c = oracle.dopri_tableau()
    assert np.allclose(a.sum(1), c, atol=1e-15)
    assert np.all(np.triu(a) == 0)
    for w, order in ((b, 5), (bs, 4)):
        assert abs(w.sum() - 1) < 1e-15
        for q in range(1, order):                       # bushy trees: sum w c^q = 1/(q+1)
            assert abs(w @ c**q - 1.0 / (q + 1)) < 1e-14, (order, q)
        assert abs(w @ (a @ c) - 1 / 6) < 1e-14          # order 3
        if order >= 4:
            assert abs(w @ (c * (a @ c)) - 1 / 8) < 1e-14
            assert abs(w @ (a @ c**2) - 1 / 12) < 1e-14
            assert abs(w @ (a @ (a @ c)) - 1 / 24) < 1e-14
        if order >= 5:
            assert abs(w @ (c**2 * (a @ c)) - 1 / 10) < 1e-14
            assert abs(w @ ((a @ c) ** 2) - 1 / 20) < 1e-14
            assert abs(w @ (c * (a @ c**2)) - 1 / 15) < 1e-14
            assert abs(w @ (a @ c**3) - 1 / 20) < 1e-14
            assert abs(w @ (c * (a @ (a @ c))) - 1 / 30) < 1e-14
            assert abs(w @ (a @ (c * (a @ c))) - 1 / 40) < 1e-14
            assert abs(w @ (a @ (a @ c**2)) - 1 / 60) < 1e-14
            assert abs(w @ (a @ (a @ (a @ c))) - 1 / 120) < 1e-14
    # the pair is not trivially equal
    assert np.abs(b - bs).max() > 1e-3


def test_rhs_is_the_projected_field(oracle):
    """f(s) = (s.s) h - (s.h) s: perpendicular to every spin, equal to the
    tangent-plane projection of the field for unit spins."""
    s = inputs.random_unit_spins((3, 2, 5, 6), seed=3)
    f, h = oracle.rk_rhs(s, 1.0, 0.3, 0.1, 0.05)
    assert np.allclose(oracle.field(s, 1.0, 0.3, 0.1, 0.05), h)
    assert np.abs((f * s).sum(0)).max() < 1e-13
    sh = (s * h).sum(0)
    assert np.allclose(f, h - sh[None] * s, atol=1e-13)


def test_single_spin_fixed_steps_fifth_order(oracle):
    """Global error of fixed steps on the closed-form single-spin flow falls
    at least like h^5 (ratio >= 24 per halving; the pair's small leading
    error constant puts the coarse steps nearer h^6, ratio 64), which a
    wrong coefficient would break (order <= 4: ratio <= 16)."""
    th0, k, T = 1.0, 1.0, 2.0
    ref = np.cos(exact_theta(th0, k, T))
    errs = []
    for n in (8, 16, 32, 64):
        y, _ = oracle.dopri_fixed(single_spin(th0), 0.0, 0.0, k, 0.0, T / n, n)
        errs.append(abs(y[2, 0, 0, 0] - ref))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(24 < r < 80 for r in ratios), (errs, ratios)
    assert errs[-1] < 1e-10


def test_single_spin_error_estimate_scaling(oracle):
    """The embedded estimate |y5 - y4| of one step scales like h^5."""
    th0, k = 0.8, 0.4
    e = [oracle.dopri_fixed(single_spin(th0), 0.0, 0.0, k, 0.0, h, 1)[1] for h in (0.2, 0.1, 0.05)]
    assert 24 < e[0] / e[1] < 40 and 26 < e[1] / e[2] < 38, e


def test_single_spin_adaptive_interval(oracle):
    """Adaptive integration over T matches the closed form to the tolerance
    and reaches T exactly; looser tolerances take fewer steps."""
    th0, k, T = 1.2, 0.3, 3.0
    ref = exact_theta(th0, k, T)
    tight = oracle.rk_interval(single_spin(th0), 0.0, 0.0, k, 0.0, T, 1e-11, 1e-11, 0.01)
    loose = oracle.rk_interval(single_spin(th0), 0.0, 0.0, k, 0.0, T, 1e-5, 1e-5, 0.01)
    assert tight["ok"] and loose["ok"]
    # local tolerance 1e-5 accumulates to a global error of order 1e-4
    for r, tol in ((tight, 1e-9), (loose, 1e-3)):
        y = r["y"][:, 0, 0, 0]
        assert abs(np.linalg.norm(y) - 1) < 1e-14          # renormalised
        assert abs(np.arctan2(y[0], y[2]) - ref) < tol
    assert loose["acc"] < tight["acc"]


def test_stationary_minimum_does_not_move(oracle):
    """Uniform +z with exchange and anisotropy only is a minimum: f = 0, the
    interval is one accepted step and the state is unchanged."""
    s = np.zeros((3, 2, 4, 5))
    s[2] = 1.0
    r = oracle.rk_interval(s, 1.0, 0.0, 0.2, 0.0, 0.5, 1e-8, 1e-8, 0.1)
    assert r["ok"] and np.array_equal(r["y"], s)
    assert r["rej"] == 0


def test_damping_flow_lowers_the_energy(oracle):
    """The damping term is a gradient flow on the sphere: dE/dt = -|f|^2, so
    the energy after an interval is lower, by about T |f|^2 for small T."""
    p = (1.0, 0.3, 0.1, 0.02)
    s = inputs.random_unit_spins((3, 1, 6, 7), seed=11)
    f, _ = oracle.rk_rhs(s, *p)
    E0 = oracle.energy(s, *p)
    T = 1e-4
    r = oracle.rk_interval(s, *p, T, 1e-12, 1e-12, T)
    E1 = oracle.energy(r["y"], *p)
    assert E1 < E0
    assert abs((E0 - E1) / (T * (f * f).sum()) - 1) < 1e-3
    r2 = oracle.rk_interval(s, *p, 0.5, 1e-8, 1e-8, 0.05)
    assert oracle.energy(r2["y"], *p) < E1


def test_step_size_proposal_carries_over(oracle):
    """The proposal returned for the next interval is the controller's last
    value: restarting from it needs no rejections on a smooth problem."""
    p = (1.0, 0.3, 0.1, 0.0)
    s = inputs.random_unit_spins((3, 1, 5, 5), seed=5)
    r1 = oracle.rk_interval(s, *p, 0.6, 1e-7, 1e-7, 1.0)
    assert r1["rej"] >= 1                                # dt0 = 1 is far too long
    r2 = oracle.rk_interval(r1["y"], *p, 0.6, 1e-7, 1e-7, r1["dt"])
    assert r2["rej"] == 0


def test_iterate_rk_composes_intervals_and_reparam(oracle):
    """One string iteration = each image over T (own step proposal), then the
    arc-length reparametrisation."""
    w = inputs.WORKLOADS["bloch_32x32x1_k10"]
    s0 = inputs.build_string(dict(w, nx=10, ny=9, K=4, R=2.5))
    p = (w["J"], w["d"], w["ku"], w["D"])
    r = oracle.iterate_rk(s0, *p, 1, 0.3, 1e-6, 1e-6, 0.05)
    man = np.empty_like(s0)
    for kk in range(4):
        man[kk] = oracle.rk_interval(s0[kk], *p, 0.3, 1e-6, 1e-6, 0.05)["y"]
    expect = oracle.reparam(man)[0]
    assert r["iters"] == 1
    np.testing.assert_array_equal(r["s"], expect)


@pytest.mark.slow
def test_iterate_rk_lowers_the_path_energy(oracle):
    """Iterating relaxes the string: the mean image energy decreases."""
    w = inputs.WORKLOADS["bloch_32x32x1_k10"]
    s0 = inputs.build_string(dict(w, nx=12, ny=12, K=5, R=3.0))
    p = (w["J"], w["d"], w["ku"], w["D"])
    E0 = np.array([oracle.energy(x, *p) for x in s0])
    r = oracle.iterate_rk(s0, *p, 5, 0.2, 1e-6, 1e-6, 0.05)
    assert r["iters"] == 5 and r["E"].mean() < E0.mean()
