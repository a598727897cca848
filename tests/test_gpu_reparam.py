"""Step-2 variants on the GPU through the C ABI (Sec. III reparametrisation;
the climbing-image refinement of the saddle): natural cubic spline
interpolation and the climbing image, against the oracle's iteration with
the same options; graph replay equals eager launches; FP32 against FP64."""
import numpy as np
import pytest
import torch

from paper_1804_07135_amd import inputs, ssm

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def prob(nx, ny, nz, K, J=1.0, d=0.3, ku=0.1, D=0.01):
    return dict(nx=nx, ny=ny, nz=nz, K=K, J=J, d=d, ku=ku, D=D)


def params(p):
    return p["J"], p["d"], p["ku"], p["D"]


@pytest.mark.parametrize("spline,climb", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("shape,K", [((12, 10, 1), 6), ((9, 8, 3), 5), ((8, 7, 2), 16), ((12, 10, 1), 20)])
def test_options_match_oracle(oracle, spline, climb, shape, K):
    """FP64, 6 iterations, against the oracle at 1e-10.  K = 16 is the
    largest image count of the one-pass spline step in FP64; K = 20 takes the
    two-kernel one (second derivatives, then evaluation)."""
    nx, ny, nz = shape
    p = prob(nx, ny, nz, K, d=0.33, ku=0.12, D=0.05)
    s0 = inputs.perturb(inputs.bloch_point_string(nx, ny, nz, K, 2.5), 11)
    sm = ssm.StringMethod(p, ssm.SSM_FP64)
    sm.set_reparam(ssm.SSM_INTERP_SPLINE if spline else ssm.SSM_INTERP_LINEAR, climb)
    sm.set_string(s0)
    sm.iterate(6, 0.1)
    r = oracle.iterate_opts(s0, *params(p), 6, 0.1, spline=spline, climb=climb)
    np.testing.assert_allclose(sm.get_string().cpu().numpy(), r["s"], rtol=0, atol=TOL64)
    np.testing.assert_allclose(sm.energies().cpu().numpy(), r["E"], rtol=0, atol=TOL64 * np.abs(r["E"]).max())


@pytest.mark.parametrize("spline,climb", [(False, False), (True, True)])
@pytest.mark.parametrize("K1", [64, 65, 70])
def test_both_reduction_paths_in_one_batch_vs_oracle(oracle, spline, climb, K1):
    """A problem of K1 images (64: the most the one-workgroup reduction
    takes; 65, 70: one workgroup per image, the last one ends step 2)
    batched with one of 6 images (reduced in one workgroup, one-pass
    spline), FP64, 5 iterations: each problem's string and energies against
    the oracle at 1e-10, and bitwise equal to its run alone."""
    specs = [((8, 7, 1), K1, 3), ((9, 8, 1), 6, 4)]
    probs, strings = [], []
    for (nx, ny, nz), K, seed in specs:
        probs.append(prob(nx, ny, nz, K, d=0.33, ku=0.12, D=0.05))
        strings.append(inputs.perturb(inputs.bloch_point_string(nx, ny, nz, K, 2.0), seed))
    mode = ssm.SSM_INTERP_SPLINE if spline else ssm.SSM_INTERP_LINEAR
    sm = ssm.StringMethod(probs, ssm.SSM_FP64)
    sm.set_reparam(mode, climb)
    sm.set_string(strings)
    sm.iterate(5, 0.1)
    assert sm.check() == 0
    flat = sm.get_string().cpu().numpy()
    E = sm.energies().cpu().numpy()
    off = e0 = 0
    for p, s0 in zip(probs, strings):
        r = oracle.iterate_opts(s0, *params(p), 5, 0.1, spline=spline, climb=climb)
        n = r["s"].size
        np.testing.assert_allclose(flat[off:off + n].reshape(r["s"].shape), r["s"], rtol=0, atol=TOL64)
        np.testing.assert_allclose(E[e0:e0 + p["K"]], r["E"], rtol=0, atol=TOL64 * np.abs(r["E"]).max())
        one = ssm.StringMethod(p, ssm.SSM_FP64)
        one.set_reparam(mode, climb)
        one.set_string(s0)
        one.iterate(5, 0.1)
        assert np.array_equal(flat[off:off + n], one.get_string().cpu().numpy().ravel())
        assert np.array_equal(E[e0:e0 + p["K"]], one.energies().cpu().numpy())
        off += n
        e0 += p["K"]


@pytest.mark.parametrize("K", [24, 40])
def test_fp32_spline_paths_vs_oracle(oracle, K):
    """FP32-mixed form with the spline and the climbing image: K = 24 takes
    the one-pass spline step (up to 32 images in FP32), K = 40 the two-kernel
    one; both against the oracle run from the same FP32 string, 6 iterations
    (spins 2e-5, energies 1e-5 relative)."""
    p = prob(12, 10, 1, K, d=0.33, ku=0.12, D=0.05)
    s0 = inputs.perturb(inputs.bloch_point_string(12, 10, 1, K, 2.5), 13).astype(np.float32)
    sm = ssm.StringMethod(p, ssm.SSM_FP32_MIXED)
    sm.set_reparam(ssm.SSM_INTERP_SPLINE, True)
    sm.set_string(s0)
    sm.iterate(6, 0.1)
    assert sm.check() == 0
    r = oracle.iterate_opts(s0.astype(np.float64), *params(p), 6, 0.1, spline=True, climb=True)
    np.testing.assert_allclose(sm.get_string().cpu().numpy(), r["s"], rtol=0, atol=2e-5)
    np.testing.assert_allclose(sm.energies().cpu().numpy(), r["E"], rtol=0, atol=1e-5 * np.abs(r["E"]).max())


def test_bloch_32x32_climbing_spline_200(oracle):
    """The 32x32x1, 10-image workload for 200 iterations with the climbing
    image and the spline: FP64 GPU equals the oracle; barrier and its image."""
    w = inputs.WORKLOADS["bloch_32x32x1_k10"]
    p = prob(w["nx"], w["ny"], w["nz"], w["K"], w["J"], w["d"], w["ku"], w["D"])
    s0 = inputs.build_string(w)
    sm = ssm.StringMethod(p, ssm.SSM_FP64)
    sm.set_reparam(ssm.SSM_INTERP_SPLINE, True)
    sm.set_string(s0)
    sm.iterate(w["iters"], w["tau"])
    r = oracle.iterate_opts(s0, *params(p), w["iters"], w["tau"], spline=True, climb=True)
    np.testing.assert_allclose(sm.get_string().cpu().numpy(), r["s"], rtol=0, atol=TOL64)
    B, km = oracle.barrier(r["E"])
    bar = sm.barrier().cpu().numpy()[0]
    assert abs(bar[0] - B) <= TOL64 * max(1.0, abs(B)) and int(bar[1]) == km


def test_graph_equals_eager_with_options():
    w = inputs.WORKLOADS["bloch_32x32x1_k10"]
    p = prob(20, 18, 2, 7, w["J"], w["d"], w["ku"], w["D"])
    s0 = inputs.build_string(dict(w, nx=20, ny=18, nz=2, K=7, R=3.0))
    out = []
    for chunk in (0, 5):
        sm = ssm.StringMethod(p, ssm.SSM_FP64)
        sm.set_options(check_every=10, graph_chunk=chunk)
        sm.set_reparam(ssm.SSM_INTERP_SPLINE, True)
        sm.set_string(s0)
        sm.iterate(15, 0.1)
        out.append(sm.get_string())
    assert torch.equal(out[0], out[1])


def test_fp32_climbing_spline_barrier_vs_fp64():
    w = inputs.WORKLOADS["boundary_64x64x1_k20"]
    p = prob(w["nx"], w["ny"], w["nz"], w["K"], w["J"], w["d"], w["ku"], w["D"])
    s0 = inputs.build_string(w)
    res = {}
    for prec in (ssm.SSM_FP64, ssm.SSM_FP32_MIXED):
        sm = ssm.StringMethod(p, prec)
        sm.set_options(10, 20)
        sm.set_reparam(ssm.SSM_INTERP_SPLINE, True)
        sm.set_string(s0)
        sm.iterate(w["iters"], w["tau"])
        assert sm.check() == 0
        res[prec] = sm.barrier().cpu().numpy()[0][0]
    assert abs(res[ssm.SSM_FP32_MIXED] - res[ssm.SSM_FP64]) <= 1e-4 * abs(res[ssm.SSM_FP64])


def test_spline_with_integrator_and_climbing_rules():
    """The spline also serves the adaptive integrator; the climbing image
    needs the explicit step."""
    p = prob(10, 9, 1, 5)
    s0 = inputs.perturb(inputs.bloch_point_string(10, 9, 1, 5, 2.5), 2)
    sm = ssm.StringMethod(p, ssm.SSM_FP64, with_rk=True)
    sm.set_integrator(ssm.SSM_STEP_DOPRI54, 1e-6, 1e-6, 0.05)
    sm.set_reparam(ssm.SSM_INTERP_SPLINE, False)
    sm.set_string(s0)
    sm.iterate(3, 0.3)
    assert sm.check() == 0
    sm.set_reparam(ssm.SSM_INTERP_LINEAR, True)
    with pytest.raises(ssm.SSMError) as e:
        sm.iterate(1, 0.3)
    assert e.value.status == ssm.SSM_EUNSUPPORTED
    with pytest.raises(ssm.SSMError):
        sm.set_reparam(5, False)
