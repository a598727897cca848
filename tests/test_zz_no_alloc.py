"""ssm_eval_noalloc (the allocation-free evaluation) against ssm_eval of a
context over a workspace (the existing entry point, same kernels): fields,
energies and term energies of every image, in both precisions, on two calls
in a row, the second with a smaller lattice and fewer images, then a third
with the first layout and new parameters (the tables are rebuilt, and the
parameters travel with every call).  Sizes beyond the fixed scratch are
refused before anything runs."""
import numpy as np
import pytest
import torch

from paper_1804_07135_amd import inputs, ssm

pytestmark = pytest.mark.gpu


def run_noalloc(problems, precision, s):
    dt = torch.float64 if precision == ssm.SSM_FP64 else torch.float32
    n_img = sum(p["K"] for p in problems)
    spins = torch.tensor(np.concatenate([x.ravel() for x in s]), dtype=dt, device="cuda")
    h = torch.empty_like(spins)
    E = torch.empty(n_img, dtype=torch.float64, device="cuda")
    T = torch.empty((n_img, 4), dtype=torch.float64, device="cuda")
    ssm.ssm_eval_noalloc(problems, precision, spins, h, E, T)
    torch.cuda.synchronize()
    return h.cpu().numpy(), E.cpu().numpy(), T.cpu().numpy()


def run_context(problems, precision, s):
    sm = ssm.StringMethod(problems, precision)
    flat = np.concatenate([x.ravel() for x in s])
    E, h, T = sm.eval(flat)
    return h.cpu().numpy().ravel(), E.cpu().numpy(), T.cpu().numpy()


def check_same(a, b, precision):
    ha, Ea, Ta = a
    hb, Eb, Tb = b
    tol = 1e-10 if precision == ssm.SSM_FP64 else 1e-5
    assert np.abs(ha - hb).max() <= tol * np.abs(hb).max()
    assert np.abs(Ea - Eb).max() <= 1e-10 * np.abs(Eb).max()
    assert np.abs(Ta - Tb).max() <= 1e-10 * np.abs(Tb).max()


@pytest.mark.parametrize("precision", [ssm.SSM_FP64, ssm.SSM_FP32_MIXED])
def test_noalloc_equals_context_eval(precision):
    big = [dict(nx=40, ny=33, nz=2, K=5, J=1.0, d=0.3, ku=0.1, D=0.02),
           dict(nx=17, ny=24, nz=2, K=3, J=0.8, d=0.2, ku=0.05, D=0.01)]
    small = [dict(nx=12, ny=9, nz=1, K=3, J=1.1, d=0.25, ku=0.2, D=0.03)]
    sb = [inputs.perturb(inputs.bloch_point_string(p["nx"], p["ny"], p["nz"], p["K"], 4.0), 5 + i)
          for i, p in enumerate(big)]
    ss = [inputs.perturb(inputs.bloch_point_string(12, 9, 1, 3, 2.0), 9)]
    r1 = run_noalloc(big, precision, sb)
    check_same(r1, run_context(big, precision, sb), precision)
    # second call, smaller input: new tables in the same scratch
    r2 = run_noalloc(small, precision, ss)
    check_same(r2, run_context(small, precision, ss), precision)
    # the first layout again with other parameters
    big2 = [dict(p, d=p["d"] + 0.05, D=p["D"] * 2) for p in big]
    r3 = run_noalloc(big2, precision, sb)
    check_same(r3, run_context(big2, precision, sb), precision)
    assert np.abs(r3[1] - r1[1]).max() > 0  # the parameters did change the result


def test_noalloc_refuses_sizes_beyond_its_scratch():
    p = [dict(nx=256, ny=256, nz=8, K=48, J=1.0, d=0.3, ku=0.1, D=0.02)]
    spins = torch.zeros(8, dtype=torch.float32, device="cuda")  # never read: refused first
    E = torch.zeros(48, dtype=torch.float64, device="cuda")
    with pytest.raises(ssm.SSMError) as e:
        ssm.ssm_eval_noalloc(p, ssm.SSM_FP32_MIXED, spins, None, E, None)
    assert e.value.status == ssm.SSM_EUNSUPPORTED
    assert "scratch" in ssm.ssm_last_error()
