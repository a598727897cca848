"""Python binding of libssm.so (include/ssm.h), argument marshalling only.

Device memory and streams come from PyTorch; every step of the method runs in
the library's HIP kernels.  The functions ssm_* mirror the C ABI one to one
(raising SSMError on a non-zero status); StringMethod bundles a context with
its workspace; SpinEnergy is the autograd form of the energy.

There is no fallback: if libssm.so is missing or no GPU is present, these
functions raise.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssm.so")

SSM_OK = 0
SSM_EINVAL = -1
SSM_ESTATE = -2
SSM_EHIP = -3
SSM_ENONFINITE = -4
SSM_EUNSUPPORTED = -5
SSM_FP64 = 0
SSM_FP32_MIXED = 1
SSM_WITH_RK = 0x100
SSM_STEP_EULER = 0
SSM_STEP_DOPRI54 = 1
SSM_INTERP_LINEAR = 0
SSM_INTERP_SPLINE = 1
SSM_N_KERNELS = 13
SSM_FLAG_NONFINITE_ENERGY = 1
SSM_FLAG_ZERO_NORM_SPIN = 2
SSM_FLAG_NONFINITE_SPIN = 4
SSM_FLAG_RK_ERROR = 8
SSM_NOALLOC_SCRATCH_MIB = 64
FLAG_NONFINITE_ENERGY = 1
FLAG_ZERO_NORM_SPIN = 2
FLAG_NONFINITE_SPIN = 4
FLAG_RK_ERROR = 8

# every exported entry point of include/ssm.h
ABI_SYMBOLS = [
    "ssm_version", "ssm_workspace_size", "ssm_create", "ssm_destroy", "ssm_set_params",
    "ssm_set_string", "ssm_get_string", "ssm_iterate", "ssm_eval", "ssm_get_energies",
    "ssm_get_fields", "ssm_get_tangents", "ssm_get_barrier", "ssm_set_options", "ssm_autotune",
    "ssm_check", "ssm_last_error", "ssm_profile", "ssm_profile_read", "ssm_kernel_name",
    "ssm_set_integrator", "ssm_get_rk_stats", "ssm_llg", "ssm_set_reparam", "ssm_eval_noalloc",
]


class SSMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ssm status {status}: {msg}")
        self.status = status


class ssm_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_images", ctypes.c_int32), ("J", ctypes.c_double), ("d", ctypes.c_double),
                ("ku", ctypes.c_double), ("dip", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_dbl = ctypes.c_double


def load():
    """Load libssm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1804_07135_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "ssm_version": (_i32, []),
        "ssm_workspace_size": (_i32, [ctypes.POINTER(ssm_problem), _i32, _i32, ctypes.POINTER(ctypes.c_size_t)]),
        "ssm_create": (_i32, [ctypes.POINTER(ssm_problem), _i32, _i32, _vp, ctypes.c_size_t, _vp,
                              ctypes.POINTER(_vp)]),
        "ssm_destroy": (_i32, [_vp]),
        "ssm_set_params": (_i32, [_vp, _i32, _dbl, _dbl, _dbl, _dbl]),
        "ssm_set_string": (_i32, [_vp, _vp]),
        "ssm_get_string": (_i32, [_vp, _vp]),
        "ssm_iterate": (_i32, [_vp, _i32, _dbl, _dbl, _vp]),
        "ssm_eval": (_i32, [_vp, _vp, _vp, _vp, _vp]),
        "ssm_get_energies": (_i32, [_vp, _vp]),
        "ssm_get_fields": (_i32, [_vp, _vp]),
        "ssm_get_tangents": (_i32, [_vp, _vp, _vp]),
        "ssm_get_barrier": (_i32, [_vp, _vp]),
        "ssm_set_options": (_i32, [_vp, _i32, _i32]),
        "ssm_autotune": (_i32, [_vp, ctypes.c_char_p]),
        "ssm_check": (_i32, [_vp, ctypes.POINTER(_i32)]),
        "ssm_last_error": (ctypes.c_char_p, [_vp]),
        "ssm_profile": (_i32, [_vp, _i32]),
        "ssm_profile_read": (_i32, [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_i32)]),
        "ssm_kernel_name": (ctypes.c_char_p, [_i32]),
        "ssm_set_integrator": (_i32, [_vp, _i32, _dbl, _dbl, _dbl]),
        "ssm_get_rk_stats": (_i32, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
        "ssm_llg": (_i32, [_vp, _dbl, _dbl]),
        "ssm_set_reparam": (_i32, [_vp, _i32, _i32]),
        "ssm_eval_noalloc": (_i32, [ctypes.POINTER(ssm_problem), _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st, ctx=None):
    if st != SSM_OK:
        msg = load().ssm_last_error(ctx).decode(errors="replace")
        raise SSMError(st, msg)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _problems(problems):
    arr = (ssm_problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = ssm_problem(int(p["nx"]), int(p["ny"]), int(p["nz"]), int(p["K"]), float(p["J"]),
                             float(p["d"]), float(p["ku"]), float(p["D"]))
    return arr


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# one function per ABI entry point
# ---------------------------------------------------------------------------
def ssm_version():
    return load().ssm_version()


def ssm_kernel_name(i):
    r = load().ssm_kernel_name(i)
    return r.decode() if r else None


def ssm_last_error(ctx=None):
    return load().ssm_last_error(ctx).decode(errors="replace")


def ssm_workspace_size(problems, precision):
    arr = _problems(problems)
    n = ctypes.c_size_t(0)
    _check(load().ssm_workspace_size(arr, len(problems), precision, ctypes.byref(n)))
    return n.value


def ssm_create(problems, precision, workspace, stream=None):
    arr = _problems(problems)
    ctx = ctypes.c_void_p()
    _check(load().ssm_create(arr, len(problems), precision, _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream_handle(stream),
                             ctypes.byref(ctx)))
    return ctx


def ssm_destroy(ctx):
    _check(load().ssm_destroy(ctx), ctx)


def ssm_set_params(ctx, problem, J, d, ku, dip):
    _check(load().ssm_set_params(ctx, problem, J, d, ku, dip), ctx)


def ssm_set_string(ctx, spins):
    _check(load().ssm_set_string(ctx, _ptr(spins)), ctx)


def ssm_get_string(ctx, out):
    _check(load().ssm_get_string(ctx, _ptr(out)), ctx)


def ssm_iterate(ctx, max_iter, tau, tol_force=0.0, iters_out=None):
    _check(load().ssm_iterate(ctx, int(max_iter), float(tau), float(tol_force), _ptr(iters_out)), ctx)


def ssm_eval(ctx, spins=None, field=None, energy=None, terms=None):
    _check(load().ssm_eval(ctx, _ptr(spins), _ptr(field), _ptr(energy), _ptr(terms)), ctx)


def ssm_eval_noalloc(problems, precision, spins, field=None, energy=None, terms=None, stream=None):
    """Field/energy evaluation through the library's fixed device scratch (no
    context, no workspace, no device allocation)."""
    arr = _problems(problems)
    _check(load().ssm_eval_noalloc(arr, len(problems), int(precision), _ptr(spins), _ptr(field), _ptr(energy),
                                   _ptr(terms), _stream_handle(stream)))


def ssm_get_energies(ctx, out):
    _check(load().ssm_get_energies(ctx, _ptr(out)), ctx)


def ssm_get_fields(ctx, out):
    _check(load().ssm_get_fields(ctx, _ptr(out)), ctx)


def ssm_get_tangents(ctx, tangent=None, force_norm=None):
    _check(load().ssm_get_tangents(ctx, _ptr(tangent), _ptr(force_norm)), ctx)


def ssm_get_barrier(ctx, out):
    _check(load().ssm_get_barrier(ctx, _ptr(out)), ctx)


def ssm_set_options(ctx, check_every=10, graph_chunk=0):
    _check(load().ssm_set_options(ctx, int(check_every), int(graph_chunk)), ctx)


def ssm_autotune(ctx, cache_path=None):
    _check(load().ssm_autotune(ctx, cache_path.encode() if cache_path else None), ctx)


def ssm_set_integrator(ctx, method, rtol=1e-6, atol=1e-6, dt0=0.1):
    _check(load().ssm_set_integrator(ctx, int(method), float(rtol), float(atol), float(dt0)), ctx)


def ssm_set_reparam(ctx, interp=SSM_INTERP_LINEAR, climbing=False):
    _check(load().ssm_set_reparam(ctx, int(interp), 1 if climbing else 0), ctx)


def ssm_llg(ctx, t_total, alpha):
    _check(load().ssm_llg(ctx, float(t_total), float(alpha)), ctx)


def ssm_get_rk_stats(ctx, counts=None, dt=None):
    n = ctypes.c_int64(0)
    _check(load().ssm_get_rk_stats(ctx, _ptr(counts), _ptr(dt), ctypes.byref(n)), ctx)
    return n.value


def ssm_check(ctx):
    f = _i32(0)
    st = load().ssm_check(ctx, ctypes.byref(f))
    if st not in (SSM_OK, SSM_ENONFINITE):
        _check(st, ctx)
    return f.value


def ssm_profile(ctx, enable=True):
    _check(load().ssm_profile(ctx, 1 if enable else 0), ctx)


def ssm_profile_read(ctx):
    ms = (_dbl * SSM_N_KERNELS)()
    cnt = (_i32 * SSM_N_KERNELS)()
    _check(load().ssm_profile_read(ctx, ms, cnt), ctx)
    return list(ms), list(cnt)


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
class StringMethod:
    """A context plus its workspace for one or more problems.

    problems: dicts with nx, ny, nz, K, J, d, ku, D.  precision: SSM_FP64 or
    SSM_FP32_MIXED; with_rk reserves the adaptive integrator's workspace.
    Strings are torch tensors of shape [sum K, 3, nz, ny, nx] (a single
    problem) or flat [sum K*3*N] (any batch)."""

    def __init__(self, problems, precision=SSM_FP64, device="cuda", stream=None, with_rk=False):
        if isinstance(problems, dict):
            problems = [problems]
        self.problems = [dict(p) for p in problems]
        self.precision = precision
        self.dtype = torch.float64 if precision == SSM_FP64 else torch.float32
        self.device = torch.device(device)
        self.stream = stream
        flags = precision | (SSM_WITH_RK if with_rk else 0)
        nbytes = ssm_workspace_size(self.problems, flags)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.ctx = ssm_create(self.problems, flags, self._ws, stream)
        self.n_img = sum(int(p["K"]) for p in self.problems)
        self.sizes = [int(p["K"]) * 3 * int(p["nx"]) * int(p["ny"]) * int(p["nz"]) for p in self.problems]
        self.n_spin = sum(self.sizes)

    def close(self):
        if self.ctx is not None:
            ssm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self):
        if len(self.problems) == 1:
            p = self.problems[0]
            return (int(p["K"]), 3, int(p["nz"]), int(p["ny"]), int(p["nx"]))
        return (self.n_spin,)

    def _dev(self, a):
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=self.dtype).contiguous()

    def set_string(self, spins):
        if isinstance(spins, (list, tuple)):
            spins = np.concatenate([np.asarray(s, dtype=np.float64).ravel() for s in spins])
        t = self._dev(spins)
        if t.numel() != self.n_spin:
            raise ValueError(f"string has {t.numel()} values, expected {self.n_spin}")
        self._string_keepalive = t
        ssm_set_string(self.ctx, t)

    def get_string(self):
        out = torch.empty(self._shape(), dtype=self.dtype, device=self.device)
        ssm_get_string(self.ctx, out)
        return out

    def set_params(self, problem, J, d, ku, D):
        ssm_set_params(self.ctx, problem, J, d, ku, D)
        self.problems[problem].update(J=J, d=d, ku=ku, D=D)

    def iterate(self, max_iter, tau, tol_force=0.0):
        it = torch.zeros(len(self.problems), dtype=torch.int32, device=self.device)
        ssm_iterate(self.ctx, max_iter, tau, tol_force, it)
        return it

    def energies(self):
        out = torch.empty(self.n_img, dtype=torch.float64, device=self.device)
        ssm_get_energies(self.ctx, out)
        return out

    def fields(self):
        out = torch.empty(self._shape(), dtype=self.dtype, device=self.device)
        ssm_get_fields(self.ctx, out)
        return out

    def tangents(self):
        t = torch.empty(self._shape(), dtype=self.dtype, device=self.device)
        n = torch.empty(len(self.problems), dtype=torch.float64, device=self.device)
        ssm_get_tangents(self.ctx, t, n)
        return t, n

    def barrier(self):
        out = torch.empty((len(self.problems), 6), dtype=torch.float64, device=self.device)
        ssm_get_barrier(self.ctx, out)
        return out

    def eval(self, spins=None, want_field=True, want_terms=True):
        E = torch.empty(self.n_img, dtype=torch.float64, device=self.device)
        T = torch.empty((self.n_img, 4), dtype=torch.float64, device=self.device) if want_terms else None
        h = torch.empty(self._shape(), dtype=self.dtype, device=self.device) if want_field else None
        s = None
        if spins is not None:
            s = self._dev(spins)
            if s.numel() != self.n_spin:
                raise ValueError("string size mismatch")
        ssm_eval(self.ctx, s, h, E, T)
        return E, h, T

    def check(self):
        return ssm_check(self.ctx)

    def set_integrator(self, method, rtol=1e-6, atol=1e-6, dt0=0.1):
        """Step 1 of iterate(): SSM_STEP_EULER (tau = step) or SSM_STEP_DOPRI54
        (tau = interval of the adaptive Dormand-Prince integration)."""
        ssm_set_integrator(self.ctx, method, rtol, atol, dt0)

    def set_reparam(self, interp=SSM_INTERP_LINEAR, climbing=False):
        """Step 2 of iterate(): linear or natural-cubic-spline interpolation,
        optionally with a climbing image."""
        ssm_set_reparam(self.ctx, interp, climbing)

    def llg(self, t_total, alpha):
        """Evolve every image by the LLG equation (eq. (9)) over t_total with the
        adaptive integrator (set_integrator's tolerances); no reparametrisation."""
        ssm_llg(self.ctx, t_total, alpha)

    def rk_stats(self):
        """(accepted/rejected steps per image [sum K, 2], step proposals [sum K],
        field evaluations of the whole batch)."""
        counts = torch.zeros((self.n_img, 2), dtype=torch.int32, device=self.device)
        dt = torch.zeros(self.n_img, dtype=torch.float64, device=self.device)
        n = ssm_get_rk_stats(self.ctx, counts, dt)
        return counts, dt, n

    def set_options(self, check_every=10, graph_chunk=0):
        ssm_set_options(self.ctx, check_every, graph_chunk)

    def autotune(self, cache_path=None):
        ssm_autotune(self.ctx, cache_path)

    def profile(self, enable=True):
        ssm_profile(self.ctx, enable)

    def profile_read(self):
        ms, cnt = ssm_profile_read(self.ctx)
        return {ssm_kernel_name(i): (ms[i], cnt[i]) for i in range(SSM_N_KERNELS) if cnt[i]}


class SpinEnergy(torch.autograd.Function):
    """E_k(s, theta) for a single-problem StringMethod, theta = (J, d, ku, D).

    Forward: the library's field/energy evaluation (eqs. (2)-(8)).  Backward:
    dE_k/ds = -h_k (the field is minus the unconstrained gradient, eq. (2))
    and dE_k/dtheta = T_theta,k, because eq. (1) is linear in each parameter.
    """

    @staticmethod
    def forward(ctx, s, theta, sm):
        if len(sm.problems) != 1:
            raise ValueError("SpinEnergy needs a single-problem StringMethod")
        th = theta.detach().to("cpu", torch.float64)
        sm.set_params(0, float(th[0]), float(th[1]), float(th[2]), float(th[3]))
        E, h, T = sm.eval(s.detach(), want_field=True, want_terms=True)
        ctx.save_for_backward(h, T)
        ctx.sdtype = s.dtype
        ctx.tdtype = theta.dtype
        ctx.tdevice = theta.device
        return E

    @staticmethod
    def backward(ctx, g):
        h, T = ctx.saved_tensors
        g = g.to(torch.float64)
        K = g.shape[0]
        gs = (-g.view(K, *([1] * (h.dim() - 1))) * h.to(torch.float64)).to(ctx.sdtype)
        gt = (g[:, None] * T).sum(dim=0).to(device=ctx.tdevice, dtype=ctx.tdtype)
        return gs, gt, None


def spin_energy(s, theta, sm):
    return SpinEnergy.apply(s, theta, sm)
