"""ctypes shim over the FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg import this module; the product package never
does.  It shares no code with the HIP path.

Arrays are numpy float64 in the spin layout [3][nz][ny][nx] per image
(images stacked as [K][3][nz][ny][nx]); see oracle.c for the conventions and
the passage of the paper each function follows.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force=False):
    """Compile liboracle.so with gcc + OpenMP (plain -O2, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_version.restype = _i
        lib.oracle_energy_terms.argtypes = [_i, _i, _i, _p, _p]
        lib.oracle_energy.argtypes = [_i, _i, _i, _d, _d, _d, _d, _p]
        lib.oracle_energy.restype = _d
        lib.oracle_field.argtypes = [_i, _i, _i, _d, _d, _d, _d, _p, _p]
        lib.oracle_field_at.argtypes = [_i, _i, _i, _d, _d, _d, _d, _p, _p, _i64, _p]
        lib.oracle_energy_from_field.argtypes = [_i64, _p, _p]
        lib.oracle_energy_from_field.restype = _d
        lib.oracle_step.argtypes = [_i64, _i, _p, _p, _d, _p]
        lib.oracle_reparam.argtypes = [_i, _i64, _p, _p, _p, _p, _p]
        lib.oracle_reparam.restype = _i
        lib.oracle_force_norm.argtypes = [_i, _i64, _p, _p, _p]
        lib.oracle_force_norm.restype = _d
        lib.oracle_iterate.argtypes = [_i, _i, _i, _d, _d, _d, _d, _i, _i, _d, _d, _i,
                                       _p, _p, _p, _p]
        lib.oracle_iterate.restype = _i
        lib.oracle_dopri_tableau.argtypes = [_p, _p, _p, _p]
        lib.oracle_rk_rhs.argtypes = [_i, _i, _i, _d, _d, _d, _d, _p, _p, _p]
        lib.oracle_dopri_fixed.argtypes = [_i, _i, _i, _d, _d, _d, _d, _p, _d, _i]
        lib.oracle_dopri_fixed.restype = _d
        lib.oracle_rk_interval.argtypes = [_i, _i, _i, _d, _d, _d, _d, _p, _d, _d, _d, _p, _p, _p, _i]
        lib.oracle_rk_interval.restype = _i
        lib.oracle_iterate_rk.argtypes = [_i, _i, _i, _d, _d, _d, _d, _i, _i, _d, _d, _d, _d, _i,
                                          _p, _p, _p, _p, _p, _p]
        lib.oracle_iterate_rk.restype = _i
        lib.oracle_llg_rhs.argtypes = [_i, _i, _i, _d, _d, _d, _d, _d, _d, _p, _p, _p]
        lib.oracle_llg_interval.argtypes = [_i, _i, _i, _d, _d, _d, _d, _d, _d, _p, _d, _d, _d, _p, _p, _p, _i]
        lib.oracle_llg_interval.restype = _i
        lib.oracle_spline_eval.argtypes = [_i, _p, _p, _i, _p, _p]
        lib.oracle_spline_eval.restype = _i
        lib.oracle_climb_step.argtypes = [_i64, _p, _p, _p, _p, _d, _p]
        lib.oracle_reparam_opts.argtypes = [_i, _i64, _p, _p, _p, _p, _p, _i, _i]
        lib.oracle_reparam_opts.restype = _i
        lib.oracle_iterate_opts.argtypes = [_i, _i, _i, _d, _d, _d, _d, _i, _i, _d, _d, _i, _i, _i,
                                            _p, _p, _p, _p]
        lib.oracle_iterate_opts.restype = _i
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_p)


def _dims(s):
    """(nx, ny, nz) of an image array shaped [3, nz, ny, nx]."""
    return s.shape[-1], s.shape[-2], s.shape[-3]


def energy_terms(s):
    """Unit-parameter term sums (T_J, T_d, T_k, T_D) of eq. (1) for one image."""
    s = _f64(s)
    nx, ny, nz = _dims(s)
    T = np.zeros(4)
    _load().oracle_energy_terms(nx, ny, nz, _ptr(s), _ptr(T))
    return T


def energy(s, J, d, k, D):
    """Total energy of one image by the bond and pair sums of eq. (1)."""
    s = _f64(s)
    nx, ny, nz = _dims(s)
    return _load().oracle_energy(nx, ny, nz, J, d, k, D, _ptr(s))


def field(s, J, d, k, D):
    """h = -dE/ds for one image [3,nz,ny,nx] (eqs. (2)-(7)), direct dipole sum."""
    s = _f64(s)
    nx, ny, nz = _dims(s)
    h = np.empty_like(s)
    _load().oracle_field(nx, ny, nz, J, d, k, D, _ptr(s), _ptr(h))
    return h


def field_at(s, J, d, k, D, sites):
    """h at flat site indices `sites` of one image; returns [len(sites), 3]."""
    s = _f64(s)
    nx, ny, nz = _dims(s)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 3))
    _load().oracle_field_at(nx, ny, nz, J, d, k, D, _ptr(s), _ptr(sites), len(sites), _ptr(out))
    return out


def energy_from_field(s, h):
    """E = -1/2 sum h.s (eq. (8)) for one image."""
    s = _f64(s)
    h = _f64(h)
    N = s.size // 3
    return _load().oracle_energy_from_field(N, _ptr(s), _ptr(h))


def step(s, h, tau):
    """Descent step + renormalisation for a string [K,3,nz,ny,nx] (eq. (10))."""
    s = _f64(s)
    h = _f64(h)
    K = s.shape[0]
    N = s[0].size // 3
    out = np.empty_like(s)
    _load().oracle_step(N, K, _ptr(s), _ptr(h), tau, _ptr(out))
    return out


def reparam(s_star):
    """Arc-length reparametrisation (eqs. (11)-(12)).

    Returns (s_new, alpha_star, j, w, applied)."""
    s_star = _f64(s_star)
    K = s_star.shape[0]
    N = s_star[0].size // 3
    out = np.empty_like(s_star)
    al = np.zeros(K)
    jj = np.zeros(K, dtype=np.int32)
    w = np.zeros(K)
    applied = _load().oracle_reparam(K, N, _ptr(s_star), _ptr(out), _ptr(al), _ptr(jj), _ptr(w))
    return out, al, jj, w, bool(applied)


def force_norm(s, h, want_tangents=False):
    """Perpendicular-force norm of a string; optionally its tangents."""
    s = _f64(s)
    h = _f64(h)
    K = s.shape[0]
    N = s[0].size // 3
    t = np.empty_like(s) if want_tangents else None
    n = _load().oracle_force_norm(K, N, _ptr(s), _ptr(h), _ptr(t) if want_tangents else None)
    return (n, t) if want_tangents else n


def iterate(s, J, d, k, D, max_iter, tau, tol=0.0, every=1, want_fields=False):
    """Run the string method (Sec. III) on a copy of s [K,3,nz,ny,nx].

    Returns dict(s=final string, E=final energies, iters=iterations done,
    force=perpendicular-force norm of the final string, h=fields or None)."""
    s = _f64(s).copy()
    K = s.shape[0]
    nx, ny, nz = _dims(s[0])
    E = np.zeros(K)
    h = np.empty_like(s) if want_fields else None
    fn = np.zeros(1)
    it = _load().oracle_iterate(nx, ny, nz, J, d, k, D, K, max_iter, tau, tol, every,
                                _ptr(s), _ptr(E), _ptr(h) if want_fields else None, _ptr(fn))
    return dict(s=s, E=E, iters=it, force=float(fn[0]), h=h)


def barrier(E):
    """B = max_k E_k - E_0 and the smallest index attaining the max (Sec. III)."""
    E = np.asarray(E, dtype=np.float64)
    km = int(np.argmax(E))
    return float(E[km] - E[0]), km


def dopri_tableau():
    """Dormand-Prince 5(4) coefficients used by the integrator: (A[7,7], b, b*, c)."""
    a = np.zeros(49)
    b = np.zeros(7)
    bs = np.zeros(7)
    c = np.zeros(7)
    _load().oracle_dopri_tableau(_ptr(a), _ptr(b), _ptr(bs), _ptr(c))
    return a.reshape(7, 7), b, bs, c


def rk_rhs(s, J, d, k, D):
    """Damping-only right-hand side f(s) = (s.s) h - (s.h) s of one image; returns (f, h)."""
    s = _f64(s)
    nx, ny, nz = _dims(s)
    f = np.empty_like(s)
    h = np.empty_like(s)
    _load().oracle_rk_rhs(nx, ny, nz, J, d, k, D, _ptr(s), _ptr(f), _ptr(h))
    return f, h


def dopri_fixed(s, J, d, k, D, hs, n):
    """n fixed Dormand-Prince steps of size hs on a copy of one image (no
    renormalisation); returns (y, RMS of the last step's error estimate)."""
    y = _f64(s).copy()
    nx, ny, nz = _dims(y)
    err = _load().oracle_dopri_fixed(nx, ny, nz, J, d, k, D, _ptr(y), hs, n)
    return y, err


def rk_interval(s, J, d, k, D, T, rtol, atol, dt0, max_steps=1000000):
    """Evolve one image over T with step control (copy); returns dict(y, dt, acc, rej, ok)."""
    y = _f64(s).copy()
    nx, ny, nz = _dims(y)
    dtp = np.array([dt0], dtype=np.float64)
    acc = np.zeros(1, dtype=np.int64)
    rej = np.zeros(1, dtype=np.int64)
    rc = _load().oracle_rk_interval(nx, ny, nz, J, d, k, D, _ptr(y), T, rtol, atol, _ptr(dtp),
                                    _ptr(acc), _ptr(rej), max_steps)
    return dict(y=y, dt=float(dtp[0]), acc=int(acc[0]), rej=int(rej[0]), ok=rc == 0)


def iterate_rk(s, J, d, k, D, max_iter, T, rtol, atol, dt0, tol=0.0, every=1, want_fields=False):
    """The string method with step 1 by the adaptive Dormand-Prince integrator
    over T per image.  Returns dict(s, E, iters, force, h, dt[K], stats[K,2])."""
    s = _f64(s).copy()
    K = s.shape[0]
    nx, ny, nz = _dims(s[0])
    E = np.zeros(K)
    h = np.empty_like(s) if want_fields else None
    fn = np.zeros(1)
    dtp = np.full(K, float(dt0))
    stats = np.zeros(2 * K, dtype=np.int64)
    it = _load().oracle_iterate_rk(nx, ny, nz, J, d, k, D, K, max_iter, T, rtol, atol, tol, every,
                                   _ptr(s), _ptr(E), _ptr(h) if want_fields else None, _ptr(fn),
                                   _ptr(dtp), _ptr(stats))
    return dict(s=s, E=E, iters=it, force=float(fn[0]), h=h, dt=dtp, stats=stats.reshape(K, 2))


def llg_coefficients(alpha):
    """(cp, cd) of eq. (9) in reduced time: 1/(1+alpha^2), alpha/(1+alpha^2)."""
    return 1.0 / (1.0 + alpha * alpha), alpha / (1.0 + alpha * alpha)


def llg_rhs(s, J, d, k, D, alpha):
    """Full LLG right-hand side of one image; returns (f, h)."""
    s = _f64(s)
    nx, ny, nz = _dims(s)
    cp, cd = llg_coefficients(alpha)
    f = np.empty_like(s)
    h = np.empty_like(s)
    _load().oracle_llg_rhs(nx, ny, nz, J, d, k, D, cp, cd, _ptr(s), _ptr(f), _ptr(h))
    return f, h


def llg_interval(s, J, d, k, D, alpha, T, rtol, atol, dt0, max_steps=1000000):
    """Evolve one image by eq. (9) over T with the adaptive Dormand-Prince pair
    (copy; renormalised at the end); returns dict(y, dt, acc, rej, ok)."""
    y = _f64(s).copy()
    nx, ny, nz = _dims(y)
    cp, cd = llg_coefficients(alpha)
    dtp = np.array([dt0], dtype=np.float64)
    acc = np.zeros(1, dtype=np.int64)
    rej = np.zeros(1, dtype=np.int64)
    rc = _load().oracle_llg_interval(nx, ny, nz, J, d, k, D, cp, cd, _ptr(y), T, rtol, atol, _ptr(dtp),
                                     _ptr(acc), _ptr(rej), max_steps)
    return dict(y=y, dt=float(dtp[0]), acc=int(acc[0]), rej=int(rej[0]), ok=rc == 0)


def spline_eval(x, f, t):
    """Natural cubic spline through (x, f) at t; returns (values, used_spline)."""
    x = _f64(x)
    f = _f64(f)
    t = _f64(t)
    out = np.empty_like(t)
    ok = _load().oracle_spline_eval(len(x), _ptr(x), _ptr(f), len(t), _ptr(t), _ptr(out))
    return out, bool(ok)


def climb_step(s_prev, s, s_next, h, tau):
    """Climbing-image step of one image (force F - 2 (F.t) t, renormalised)."""
    s_prev, s, s_next, h = (_f64(a) for a in (s_prev, s, s_next, h))
    out = np.empty_like(s)
    _load().oracle_climb_step(s.size // 3, _ptr(s_prev), _ptr(s), _ptr(s_next), _ptr(h), tau, _ptr(out))
    return out


def reparam_opts(s_star, spline=False, kci=-1):
    """Step 2 with a natural cubic spline and/or a climbing image kci (-1: none).
    Returns (s_new, alpha_star, j, w, applied)."""
    s_star = _f64(s_star)
    K = s_star.shape[0]
    N = s_star[0].size // 3
    out = np.empty_like(s_star)
    al = np.zeros(K)
    jj = np.zeros(K, dtype=np.int32)
    w = np.zeros(K)
    applied = _load().oracle_reparam_opts(K, N, _ptr(s_star), _ptr(out), _ptr(al), _ptr(jj), _ptr(w),
                                          1 if spline else 0, int(kci))
    return out, al, jj, w, bool(applied)


def iterate_opts(s, J, d, k, D, max_iter, tau, spline=False, climb=False, tol=0.0, every=1,
                 want_fields=False):
    """iterate() with the step-2 options.  Returns the same dict as iterate()."""
    s = _f64(s).copy()
    K = s.shape[0]
    nx, ny, nz = _dims(s[0])
    E = np.zeros(K)
    h = np.empty_like(s) if want_fields else None
    fn = np.zeros(1)
    it = _load().oracle_iterate_opts(nx, ny, nz, J, d, k, D, K, max_iter, tau, tol, every,
                                     1 if spline else 0, 1 if climb else 0, _ptr(s), _ptr(E),
                                     _ptr(h) if want_fields else None, _ptr(fn))
    return dict(s=s, E=E, iters=it, force=float(fn[0]), h=h)
