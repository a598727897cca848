"""SI front end and (d, k) phase-diagram driver.

The paper (Sec. IV) states its material in SI units: lattice constant
a = 0.2715 nm, moment |S| = 2.3737 mu_B, exchange J = 54.23 meV, DMI d and
anisotropy k in meV, a 112 x 112 x 1 monolayer, 60 images, and an interval
Delta t = 5e-14 s of the damping dynamics per string iteration; the
reduced gyromagnetic ratio is gamma = 2.2127615e5 m/(A s) (Sec. II.B).  The
library works in reduced units (energies in units of J, lattice constant
1, time in units of mu0 |S| / (gamma J)); this module converts between the
two and runs batched sweeps over (d, k) grids, the computation behind the
paper's phase diagrams (Fig. 3).  The damping constant alpha is not given
in the paper; it is a parameter here.

Conversions:
  d_red = d / J,  k_red = k / J,
  D_red = mu0 |S|^2 / (4 pi a^3) / J        (dipolar strength, eq. (1)),
  t0 = mu0 |S| / (gamma J)                   (time unit of eq. (9)),
  the string method's step-1 interval in its own time (damping prefactor
  alpha / (1 + alpha^2) absorbed): Delta t / t0 * alpha / (1 + alpha^2).
"""
import math
from dataclasses import dataclass

import numpy as np

MU_0 = 1.25663706212e-6         # vacuum permeability, N / A^2 (CODATA 2018)
MU_B = 9.2740100783e-24         # Bohr magneton, J / T (CODATA 2018)
EV = 1.602176634e-19            # J per eV (exact)
GAMMA = 2.2127615e5             # reduced gyromagnetic ratio, m / (A s) (Sec. II.B)


@dataclass(frozen=True)
class Material:
    """Lattice constant a (m), spin moment S (units of mu_B), exchange J (meV)."""
    a: float = 0.2715e-9
    S: float = 2.3737
    J_meV: float = 54.23

    @property
    def J_joule(self):
        return self.J_meV * 1e-3 * EV

    @property
    def moment(self):
        """|S| in A m^2."""
        return self.S * MU_B


PAPER = Material()


def dipolar_reduced(m=PAPER):
    """D = mu0 |S|^2 / (4 pi a^3) in units of J."""
    return MU_0 * m.moment ** 2 / (4.0 * math.pi * m.a ** 3) / m.J_joule


def time_unit(m=PAPER):
    """t0 = mu0 |S| / (gamma J) in seconds: the time unit of eq. (9) in reduced units."""
    return MU_0 * m.moment / (GAMMA * m.J_joule)


def interval_reduced(dt_seconds, alpha, m=PAPER):
    """Step-1 interval of the string method (damping term alone, prefactor
    alpha/(1+alpha^2) absorbed into its time) for an SI interval dt."""
    return dt_seconds / time_unit(m) * alpha / (1.0 + alpha * alpha)


def llg_time_reduced(t_seconds, m=PAPER):
    """Time argument of ssm_llg (eq. (9) in reduced time) for an SI time."""
    return t_seconds / time_unit(m)


def reduced_params(d_meV, k_meV, m=PAPER, dipolar=True):
    """Problem parameters (J, d, ku, D) in reduced units."""
    return dict(J=1.0, d=d_meV / m.J_meV, ku=k_meV / m.J_meV, D=dipolar_reduced(m) if dipolar else 0.0)


def energy_meV(E_reduced, m=PAPER):
    """Energies (barriers) from units of J to meV."""
    return np.asarray(E_reduced) * m.J_meV


def paper_problem(d_meV, k_meV, m=PAPER, n=112, K=60, dipolar=True):
    """The paper's monolayer (n x n x 1, K images) at (d, k) in meV."""
    return dict(nx=n, ny=n, nz=1, K=K, **reduced_params(d_meV, k_meV, m, dipolar))


def initial_string(process, n, K, R, seed):
    """Bloch-point (shrinking skyrmion) or boundary (translated skyrmion)
    initial string of the paper's two annihilation processes (Sec. IV)."""
    from . import inputs
    if process == "bloch":
        s = inputs.bloch_point_string(n, n, 1, K, R)
    elif process == "boundary":
        s = inputs.boundary_string(n, n, 1, K, R)
    else:
        raise ValueError("process must be 'bloch' or 'boundary'")
    return inputs.perturb(s, seed)


def phase_diagram(d_meV, k_meV, process="bloch", m=PAPER, n=112, K=60, R=10.0, alpha=1.0,
                  dt_seconds=5e-14, iters=1000, tol_force=0.0, precision=None, integrator="dopri",
                  rtol=1e-5, atol=1e-5, climbing=False, spline=False, check_every=50, seed=0,
                  autotune_cache=None):
    """Annihilation barriers (meV) on the grid d_meV x k_meV (Fig. 3).

    Every grid point is one problem of a single batched context (all points
    advance together).  integrator: "dopri" evolves each image over the
    paper's interval (Delta t converted with alpha) with the adaptive
    Dormand-Prince pair; "euler" takes one explicit step of that length.
    autotune_cache: path of a tile cache; when given, the kernels' tiles are
    tuned on this context first (results then depend on the tiles only
    through the order of floating-point sums).
    Returns dict(barrier[len(d), len(k)] in meV, argmax, dB_dd and dB_dk (the
    envelope-theorem derivatives, meV per meV; NaN where the path did not
    converge), converged (final perpendicular-force norm finite and below
    tol_force), iters, force, flags (ssm_check bits of the run), context)."""
    from . import ssm
    if precision is None:
        precision = ssm.SSM_FP32_MIXED
    dd, kk = np.meshgrid(np.asarray(d_meV, float), np.asarray(k_meV, float), indexing="ij")
    probs = [paper_problem(d, k, m, n, K) for d, k in zip(dd.ravel(), kk.ravel())]
    strings = [initial_string(process, n, K, R, seed + i) for i in range(len(probs))]
    sm = ssm.StringMethod(probs, precision, with_rk=(integrator == "dopri"))
    sm.set_options(check_every=check_every, graph_chunk=check_every if integrator == "euler" else 0)
    sm.set_reparam(ssm.SSM_INTERP_SPLINE if spline else ssm.SSM_INTERP_LINEAR, climbing)
    tau = interval_reduced(dt_seconds, alpha, m)
    if integrator == "dopri":
        sm.set_integrator(ssm.SSM_STEP_DOPRI54, rtol, atol, tau / 10)
    elif integrator != "euler":
        raise ValueError("integrator must be 'dopri' or 'euler'")
    sm.set_string(strings)
    if autotune_cache is not None:
        sm.autotune(autotune_cache)
    it = sm.iterate(iters, tau, tol_force).cpu().numpy()
    bar = sm.barrier().cpu().numpy()
    _, fn = sm.tangents()
    force = fn.cpu().numpy()
    flags = sm.check()
    from .sweep import converged_mask, mask_unconverged
    conv = converged_mask(force, tol_force) & np.isfinite(bar[:, 0])
    dB = mask_unconverged(bar[:, 2:6], conv)
    shape = dd.shape
    # barrier derivatives: dB/d(d_red) * d(d_red)/d(d_meV) with d_red = d/J,
    # and B in meV = B_red * J, so dB_meV/dd_meV = dB_red/dd_red
    return dict(barrier=energy_meV(bar[:, 0]).reshape(shape), argmax=bar[:, 1].astype(int).reshape(shape),
                dB_dd=dB[:, 1].reshape(shape), dB_dk=dB[:, 2].reshape(shape), converged=conv.reshape(shape),
                iters=it.reshape(shape), force=force.reshape(shape), flags=flags, context=sm)
