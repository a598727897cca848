"""Batched parameter sweeps of the string method (one context, many points).

Every (k_u, d) point of a sweep, each with its own lattice size, is one
problem of a single context, so every kernel of an iteration covers all of
them in one launch, and iterations are replayed as a HIP graph.  The result
per point is the barrier (Sec. III: energy of the highest image relative to
the first) and its derivatives with respect to the parameters of eq. (1) by
the envelope theorem: at a converged path dB/dtheta = T_theta(k*) - T_theta(0),
because the energy is linear in every parameter.
"""
import numpy as np
import torch

from . import inputs, ssm


def sweep_problems(points):
    return [dict(nx=p["nx"], ny=p["ny"], nz=p["nz"], K=p["K"], J=p["J"], d=p["d"], ku=p["ku"],
                 D=p["D"]) for p in points]


def initial_strings(points):
    return [inputs.perturb(inputs.bloch_point_string(p["nx"], p["ny"], p["nz"], p["K"], p["R"]),
                           p["seed"]) for p in points]


def converged_mask(force, tol_force):
    """Points whose final perpendicular-force norm is finite and below
    tol_force (none when tol_force is 0: a fixed iteration count proves no
    convergence)."""
    force = np.asarray(force, dtype=np.float64)
    return np.isfinite(force) & (force < tol_force) if tol_force > 0 else np.zeros(force.shape, bool)


def mask_unconverged(dB, converged):
    """Envelope derivatives hold only at a converged path (Sec. III): NaN
    elsewhere."""
    dB = np.array(dB, dtype=np.float64, copy=True)
    dB[~np.asarray(converged, bool)] = np.nan
    return dB


def run_sweep(points, precision=ssm.SSM_FP32_MIXED, max_iter=20000, tau=0.1, tol_force=1e-4,
              check_every=50, graph_chunk=50, autotune_cache=None, strings=None, interp=None,
              climbing=False):
    """Converge the strings of all points in one batched context.

    Returns dict(barrier[P], argmax[P], dB[P,4] (J, d, ku, dip; NaN at points
    that did not converge), converged[P], iters[P], force[P] (final
    perpendicular-force norm, inf if non-finite), flags (ssm_check bits of
    the whole run), energies (list of per-point arrays), context)."""
    sm = ssm.StringMethod(sweep_problems(points), precision)
    sm.set_options(check_every=check_every, graph_chunk=graph_chunk)
    if interp is not None or climbing:
        sm.set_reparam(ssm.SSM_INTERP_LINEAR if interp is None else interp, climbing)
    sm.set_string(strings if strings is not None else initial_strings(points))
    if autotune_cache is not None:
        sm.autotune(autotune_cache)
    iters = sm.iterate(max_iter, tau, tol_force).cpu().numpy()
    bar = sm.barrier().cpu().numpy()
    _, fn = sm.tangents()
    force = fn.cpu().numpy()
    flags = sm.check()
    E = sm.energies().cpu().numpy()
    out_E, o = [], 0
    for p in points:
        out_E.append(E[o:o + p["K"]])
        o += p["K"]
    conv = converged_mask(force, tol_force) & np.isfinite(bar[:, 0])
    return dict(barrier=bar[:, 0], argmax=bar[:, 1].astype(int), dB=mask_unconverged(bar[:, 2:6], conv),
                converged=conv, iters=iters, force=force, flags=flags, energies=out_E, context=sm)


def split_string(sm, points):
    """The converged string of every point as [K,3,nz,ny,nx] arrays."""
    flat = sm.get_string().reshape(-1)
    out, o = [], 0
    for p in points:
        n = p["K"] * 3 * p["nx"] * p["ny"] * p["nz"]
        out.append(flat[o:o + n].reshape(p["K"], 3, p["nz"], p["ny"], p["nx"]))
        o += n
    return out
