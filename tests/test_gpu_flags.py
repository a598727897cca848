"""Failure flags of ssm_check, forced from the host input: an interpolated
spin of zero norm (antiparallel sources at weight 1/2, Sec. III
interpolation guard) and a non-finite spin in the string."""
import numpy as np
import pytest

from paper_1804_07135_amd import ssm

pytestmark = pytest.mark.gpu


def one_site_string(zs):
    """K images of a 1x1x1 lattice, spin (0, 0, z_k)."""
    s = np.zeros((len(zs), 3, 1, 1, 1))
    s[:, 2, 0, 0, 0] = zs
    return s


@pytest.mark.parametrize("precision", [ssm.SSM_FP64, ssm.SSM_FP32_MIXED])
def test_zero_norm_interpolation_takes_nearer_source(precision):
    """Images +z, +z, -z with a zero step: arc lengths 0 and 2, so the middle
    target t = 1/2 sits at weight exactly 1/2 between +z and -z.  The
    interpolated spin has norm 0: the flag is raised and the spin of the
    second source (weight not below 1/2) is taken."""
    p = dict(nx=1, ny=1, nz=1, K=3, J=1.0, d=0.0, ku=0.1, D=0.0)
    sm = ssm.StringMethod(p, precision)
    sm.set_string(one_site_string([1.0, 1.0, -1.0]))
    sm.iterate(1, 0.0)
    flags = sm.check()
    assert flags & ssm.SSM_FLAG_ZERO_NORM_SPIN
    assert not flags & (ssm.SSM_FLAG_NONFINITE_ENERGY | ssm.SSM_FLAG_NONFINITE_SPIN)
    s = sm.get_string().cpu().numpy().reshape(3, 3)
    np.testing.assert_array_equal(s[1], [0.0, 0.0, -1.0])
    assert sm.check() == 0  # flags are cleared by reading them


@pytest.mark.parametrize("precision", [ssm.SSM_FP64, ssm.SSM_FP32_MIXED])
def test_nonfinite_spin_is_flagged(precision):
    p = dict(nx=6, ny=5, nz=1, K=4, J=1.0, d=0.2, ku=0.1, D=0.01)
    rng = np.random.default_rng(0)
    s = rng.standard_normal((4, 3, 1, 5, 6))
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    s[2, 0, 0, 2, 3] = np.nan
    sm = ssm.StringMethod(p, precision)
    sm.set_string(s)
    sm.iterate(1, 0.1)
    flags = sm.check()
    assert flags & ssm.SSM_FLAG_NONFINITE_ENERGY
    assert sm.check() == 0


@pytest.mark.parametrize("precision", [ssm.SSM_FP64, ssm.SSM_FP32_MIXED])
def test_nonfinite_problem_never_counts_as_converged(precision):
    """A point whose string holds a NaN spin has a non-finite force norm: with
    tol_force > 0 it must not stop as converged, the flag must be raised,
    and the sweep driver must report it unconverged with NaN envelope
    derivatives, while a finite point of the same batch converges."""
    from paper_1804_07135_amd import sweep
    pts = [dict(nx=4, ny=3, nz=1, K=3, J=1.0, d=0.0, ku=0.2, D=0.0, R=1.0, seed=1),
           dict(nx=6, ny=5, nz=1, K=4, J=1.0, d=0.2, ku=0.1, D=0.01, R=1.0, seed=2)]
    fm = np.zeros((3, 3, 1, 3, 4))
    fm[:, 2] = 1.0  # every image the +z ferromagnet: force exactly 0
    rng = np.random.default_rng(0)
    bad = rng.standard_normal((4, 3, 1, 5, 6))
    bad /= np.linalg.norm(bad, axis=1, keepdims=True)
    bad[2, 0, 0, 2, 3] = np.nan
    r = sweep.run_sweep(pts, precision=precision, max_iter=40, tau=0.1, tol_force=1e-6,
                        check_every=10, graph_chunk=10, strings=[fm, bad])
    assert r["flags"] & ssm.SSM_FLAG_NONFINITE_ENERGY
    assert np.isinf(r["force"][1]) and not r["converged"][1]
    assert int(r["iters"][1]) == 40
    assert np.all(np.isnan(r["dB"][1]))
    assert r["converged"][0] and int(r["iters"][0]) == 0
    assert np.all(np.isfinite(r["dB"][0]))


def test_fixed_iteration_sweep_reports_no_convergence():
    """tol_force = 0 (a fixed number of iterations) proves nothing about
    convergence: every point is reported unconverged, its envelope
    derivatives NaN."""
    from paper_1804_07135_amd import sweep
    pts = [dict(nx=8, ny=8, nz=1, K=4, J=1.0, d=0.3, ku=0.1, D=0.01, R=2.0, seed=3)]
    r = sweep.run_sweep(pts, precision=ssm.SSM_FP64, max_iter=5, tol_force=0.0, check_every=5,
                        graph_chunk=0)
    assert not r["converged"][0]
    assert np.all(np.isnan(r["dB"][0])) and np.isfinite(r["barrier"][0])
