"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: the FP64 path must match the oracle to 1e-10 relative (fields
normwise, energies and barriers); the FP32-mixed path to 1e-5 for fields and
1e-4 for barriers.  Inputs are seeded and synthetic.
"""
import numpy as np
import pytest
import torch

from paper_1804_07135_amd import inputs, ssm, sweep

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32_FIELD = 1e-5
TOL32_BARRIER = 1e-4


def prob(nx, ny, nz, K, J=1.0, d=0.3, ku=0.1, D=0.01):
    return dict(nx=nx, ny=ny, nz=nz, K=K, J=J, d=d, ku=ku, D=D)


def oracle_fields(oracle, s, p):
    return np.stack([oracle.field(si, p["J"], p["d"], p["ku"], p["D"]) for si in s])


def rel_field(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# ragged and power-of-two sizes; odd and even log2 transform lengths with full
# line groups (32, 128, 512 along x); 1, 2, 3-4, 5-8 and 16 layers; half
# padded lengths 3 2^a: runtime-length 768 along x, 384 along y, 48 and 96
# along y with 9-16 layers; compile-time-length 48, 96, 192 and 384 along x
# and 48, 96 and 192 along y with 1, 4 and 8 padded layers
SHAPES = [(1, 1, 1), (2, 2, 1), (5, 3, 1), (1, 6, 1), (9, 1, 1), (6, 5, 3), (7, 9, 2),
          (33, 17, 1), (16, 16, 4), (12, 10, 8), (20, 3, 5), (3, 4, 16), (32, 32, 1),
          (100, 20, 1), (300, 5, 1), (2, 64, 1), (1000, 3, 1), (40, 128, 1),
          (20, 40, 1), (70, 70, 1), (16, 150, 1), (600, 5, 1), (33, 300, 1), (5, 40, 12), (6, 70, 9),
          (150, 20, 1), (50, 90, 3), (12, 140, 5)]


@pytest.mark.parametrize("shape", SHAPES)
def test_field_energy_terms_fp64(oracle, shape):
    nx, ny, nz = shape
    p = prob(nx, ny, nz, 3, J=0.9, d=0.35, ku=0.21, D=0.13)
    s = inputs.random_unit_spins((3, 3, nz, ny, nx), seed=nx * 100 + ny * 10 + nz)
    sm = ssm.StringMethod(p, ssm.SSM_FP64)
    E, h, T = sm.eval(s)
    h = h.cpu().numpy()
    ho = oracle_fields(oracle, s, p)
    assert rel_field(h, ho) < TOL64
    To = np.stack([oracle.energy_terms(si) for si in s])
    Eo = To @ np.array([p["J"], p["d"], p["ku"], p["D"]])
    scale = np.abs(To).max() + 1e-300
    np.testing.assert_allclose(T.cpu().numpy(), To, rtol=0, atol=TOL64 * scale)
    np.testing.assert_allclose(E.cpu().numpy(), Eo, rtol=0, atol=TOL64 * (np.abs(Eo).max() + 1))


@pytest.mark.parametrize("shape", SHAPES)
def test_field_fp32_mixed(oracle, shape):
    nx, ny, nz = shape
    p = prob(nx, ny, nz, 2, J=0.9, d=0.35, ku=0.21, D=0.13)
    s = inputs.random_unit_spins((2, 3, nz, ny, nx), seed=7 + nx + ny + nz)
    s32 = s.astype(np.float32).astype(np.float64)  # the FP32 path sees rounded spins
    sm = ssm.StringMethod(p, ssm.SSM_FP32_MIXED)
    E, h, T = sm.eval(s32)
    ho = oracle_fields(oracle, s32, p)
    assert rel_field(h.cpu().numpy().astype(np.float64), ho) < TOL32_FIELD
    Eo = np.array([oracle.energy(si, p["J"], p["d"], p["ku"], p["D"]) for si in s32])
    np.testing.assert_allclose(E.cpu().numpy(), Eo, rtol=0, atol=1e-6 * (np.abs(Eo).max() + 1))


def test_padding_and_parameters_independent(oracle):
    """The same spins in batches of different lattice parameters give fields
    that scale linearly with each parameter (eq. (1) is linear in them)."""
    nx, ny, nz = 11, 7, 2
    s = inputs.random_unit_spins((2, 3, nz, ny, nx), seed=3)
    base = prob(nx, ny, nz, 2, J=0, d=0, ku=0, D=0)
    out = []
    for k in ["J", "d", "ku", "D"]:
        sm = ssm.StringMethod(dict(base, **{k: 1.0}), ssm.SSM_FP64)
        out.append(sm.eval(s)[1].cpu().numpy())
    sm = ssm.StringMethod(dict(base, J=0.7, d=-0.2, ku=0.4, D=0.05), ssm.SSM_FP64)
    h = sm.eval(s)[1].cpu().numpy()
    comb = 0.7 * out[0] - 0.2 * out[1] + 0.4 * out[2] + 0.05 * out[3]
    assert rel_field(h, comb) < TOL64


def run_both(oracle, p, s0, iters, tau=0.1, precision=ssm.SSM_FP64, graph_chunk=0):
    sm = ssm.StringMethod(p, precision)
    sm.set_options(10, graph_chunk)
    sm.set_string(s0)
    done = sm.iterate(iters, tau)
    r = oracle.iterate(s0 if precision == ssm.SSM_FP64 else s0.astype(np.float32).astype(np.float64),
                       p["J"], p["d"], p["ku"], p["D"], iters, tau, want_fields=True)
    return sm, r, int(done[0])


def test_iterate_small_3d_fp64(oracle):
    p = prob(8, 6, 3, 4, J=1.0, d=0.3, ku=0.1, D=0.05)
    s0 = inputs.perturb(inputs.bloch_point_string(8, 6, 3, 4, 2.0), 11)
    sm, r, n = run_both(oracle, p, s0, 15)
    assert n == 15
    s = sm.get_string().cpu().numpy()
    assert np.abs(s - r["s"]).max() < TOL64
    E = sm.energies().cpu().numpy()
    np.testing.assert_allclose(E, r["E"], rtol=0, atol=TOL64 * np.abs(r["E"]).max())
    assert rel_field(sm.fields().cpu().numpy(), r["h"]) < TOL64


def test_iterate_workload_32x32_fp64(oracle):
    """The 32x32x1, 10-image Bloch-point workload, full 200 iterations."""
    w = inputs.WORKLOADS["bloch_32x32x1_k10"]
    p = prob(w["nx"], w["ny"], w["nz"], w["K"], w["J"], w["d"], w["ku"], w["D"])
    s0 = inputs.build_string(w)
    sm, r, n = run_both(oracle, p, s0, w["iters"], w["tau"])
    E = sm.energies().cpu().numpy()
    np.testing.assert_allclose(E, r["E"], rtol=0, atol=TOL64 * np.abs(r["E"]).max())
    B, km = oracle.barrier(r["E"])
    bar = sm.barrier().cpu().numpy()[0]
    assert abs(bar[0] - B) <= TOL64 * abs(B)
    assert int(bar[1]) == km
    assert np.abs(sm.get_string().cpu().numpy() - r["s"]).max() < TOL64


@pytest.mark.parametrize("L", [65, 72, 96])
def test_iterate_sweep_lattices_vs_oracle(oracle, L):
    """L x L x 1 lattices of the (k_u, d) sweep that take the 96-point
    transforms (padded length 192 for 2L - 1 = 129..191): the sweep's
    Bloch-point string of 6 images, 5 iterations.  FP64: string, energies,
    barrier and argmax against the oracle at 1e-10; FP32-mixed: barrier at
    1e-4."""
    p = prob(L, L, 1, 6, J=1.0, d=0.3, ku=0.1, D=0.01)
    pt = dict(nx=L, ny=L, nz=1, K=6, R=5.0, seed=4000 + L)
    s0 = sweep.initial_strings([pt])[0]
    sm, r, n = run_both(oracle, p, s0, 5)
    assert n == 5
    assert np.abs(sm.get_string().cpu().numpy() - r["s"]).max() < TOL64
    E = sm.energies().cpu().numpy()
    np.testing.assert_allclose(E, r["E"], rtol=0, atol=TOL64 * np.abs(r["E"]).max())
    B, km = oracle.barrier(r["E"])
    bar = sm.barrier().cpu().numpy()[0]
    assert abs(bar[0] - B) <= TOL64 * abs(B)
    assert int(bar[1]) == km
    s32 = ssm.StringMethod(p, ssm.SSM_FP32_MIXED)
    s32.set_string(s0)
    s32.iterate(5, 0.1)
    assert abs(s32.barrier().cpu().numpy()[0, 0] - B) <= TOL32_BARRIER * abs(B)


def test_iterate_workload_32x32_fp32_barrier(oracle):
    w = inputs.WORKLOADS["bloch_32x32x1_k10"]
    p = prob(w["nx"], w["ny"], w["nz"], w["K"], w["J"], w["d"], w["ku"], w["D"])
    s0 = inputs.build_string(w)
    sm = ssm.StringMethod(p, ssm.SSM_FP32_MIXED)
    sm.set_string(s0)
    sm.iterate(w["iters"], w["tau"])
    r = oracle.iterate(s0, p["J"], p["d"], p["ku"], p["D"], w["iters"], w["tau"])
    B, _ = oracle.barrier(r["E"])
    bar = sm.barrier().cpu().numpy()[0]
    assert abs(bar[0] - B) <= TOL32_BARRIER * abs(B)


def test_graph_replay_matches_eager_bitwise():
    w = inputs.WORKLOADS["bloch_32x32x1_k10"]
    p = prob(w["nx"], w["ny"], w["nz"], w["K"], w["J"], w["d"], w["ku"], w["D"])
    s0 = inputs.build_string(w)
    out = []
    for chunk in (0, 4):
        sm = ssm.StringMethod(p, ssm.SSM_FP64)
        sm.set_options(10, chunk)
        sm.set_string(s0)
        sm.iterate(13, 0.1)
        out.append((sm.get_string().cpu().numpy(), sm.energies().cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_resume_is_bitwise():
    p = prob(12, 10, 1, 5)
    s0 = inputs.perturb(inputs.bloch_point_string(12, 10, 1, 5, 3.0), 5)
    sm = ssm.StringMethod(p, ssm.SSM_FP64)
    sm.set_string(s0)
    sm.iterate(10, 0.1)
    a = sm.get_string().cpu().numpy()
    sm2 = ssm.StringMethod(p, ssm.SSM_FP64)
    sm2.set_string(s0)
    sm2.iterate(5, 0.1)
    mid = sm2.get_string()
    sm3 = ssm.StringMethod(p, ssm.SSM_FP64)
    sm3.set_string(mid)
    sm3.iterate(5, 0.1)
    assert np.array_equal(a, sm3.get_string().cpu().numpy())


def test_tangents_and_force_norm(oracle):
    p = prob(9, 7, 2, 5, D=0.03)
    s0 = inputs.perturb(inputs.bloch_point_string(9, 7, 2, 5, 2.5), 21)
    sm = ssm.StringMethod(p, ssm.SSM_FP64)
    sm.set_string(s0)
    sm.eval()
    t, n = sm.tangents()
    h = oracle_fields(oracle, s0, p)
    no, to = oracle.force_norm(s0, h, want_tangents=True)
    assert abs(float(n[0]) - no) <= TOL64 * no
    assert np.abs(t.cpu().numpy() - to).max() < TOL64


def test_convergence_matches_oracle(oracle):
    p = prob(6, 6, 1, 4)
    s0 = inputs.perturb(inputs.bloch_point_string(6, 6, 1, 4, 1.5), 9)
    sm = ssm.StringMethod(p, ssm.SSM_FP64)
    sm.set_options(5, 0)
    sm.set_string(s0)
    it = int(sm.iterate(5000, 0.1, tol_force=2e-2)[0])
    r = oracle.iterate(s0, 1.0, 0.3, 0.1, 0.01, 5000, 0.1, tol=2e-2, every=5)
    assert it == r["iters"]
    np.testing.assert_allclose(sm.energies().cpu().numpy(), r["E"], rtol=0,
                               atol=TOL64 * np.abs(r["E"]).max())


def test_degenerate_string_skips_reparam(oracle):
    p = prob(5, 4, 1, 3, d=0.0, D=0.0)
    s0 = np.stack([inputs.ferromagnet(5, 4, 1)] * 3)
    sm, r, _ = run_both(oracle, p, s0, 3)
    assert np.array_equal(sm.get_string().cpu().numpy(), r["s"])
    assert sm.check() == 0


def test_two_images(oracle):
    p = prob(7, 5, 1, 2)
    s0 = inputs.perturb(inputs.bloch_point_string(7, 5, 1, 2, 2.0), 4)
    sm, r, _ = run_both(oracle, p, s0, 7)
    assert np.abs(sm.get_string().cpu().numpy() - r["s"]).max() < TOL64


@pytest.mark.parametrize("nprob", [64, 70])
def test_batch_of_many_problems_equals_separate_runs(oracle, nprob):
    """64 problems (the most one wavefront's ballot lookup serves) and 70
    (more: the workgroups find their problem by binary search), of both x
    length kinds (8, 16 and 48-point half lengths) and several image counts:
    every seventh problem's string and energies, and the last one's, bitwise
    equal to its run alone after 3 iterations, and the first and last
    against the oracle at 1e-10."""
    rng = np.random.default_rng(70)
    shapes = [(int(rng.choice([5, 9, 12, 40, 45])), int(rng.integers(3, 9)), int(rng.integers(2, 5)))
              for _ in range(nprob)]
    probs = [prob(nx, ny, 1, K, d=0.2 + 0.002 * i) for i, (nx, ny, K) in enumerate(shapes)]
    strings = [inputs.perturb(inputs.bloch_point_string(nx, ny, 1, K, 1.5), i)
               for i, (nx, ny, K) in enumerate(shapes)]
    sm = ssm.StringMethod(probs, ssm.SSM_FP64)
    sm.set_string(strings)
    sm.iterate(3, 0.1)
    flat = sm.get_string().cpu().numpy()
    E = sm.energies().cpu().numpy()
    off = e0 = 0
    for i, (p, s0) in enumerate(zip(probs, strings)):
        n = s0.size
        if i in (0, nprob - 1):
            r = oracle.iterate(s0, p["J"], p["d"], p["ku"], p["D"], 3, 0.1)
            assert np.abs(flat[off:off + n] - r["s"].ravel()).max() < TOL64
        if i % 7 == 0 or i == nprob - 1:
            one = ssm.StringMethod(p, ssm.SSM_FP64)
            one.set_string(s0)
            one.iterate(3, 0.1)
            assert np.array_equal(flat[off:off + n], one.get_string().cpu().numpy().ravel())
            assert np.array_equal(E[e0:e0 + p["K"]], one.energies().cpu().numpy())
        off += n
        e0 += p["K"]


def test_batch_equals_separate_runs():
    shapes = [(10, 9, 1, 4, 0.2), (17, 5, 1, 3, 0.3), (8, 8, 1, 5, 0.4)]
    probs = [prob(nx, ny, nz, K, d=d) for nx, ny, nz, K, d in shapes]
    strings = [inputs.perturb(inputs.bloch_point_string(nx, ny, nz, K, 2.0), i)
               for i, (nx, ny, nz, K, _) in enumerate(shapes)]
    sm = ssm.StringMethod(probs, ssm.SSM_FP64)
    sm.set_string(strings)
    sm.iterate(6, 0.1)
    flat = sm.get_string().cpu().numpy()
    E = sm.energies().cpu().numpy()
    off = e0 = 0
    for p, s0 in zip(probs, strings):
        one = ssm.StringMethod(p, ssm.SSM_FP64)
        one.set_string(s0)
        one.iterate(6, 0.1)
        a = one.get_string().cpu().numpy().ravel()
        assert np.array_equal(flat[off:off + a.size], a)
        assert np.array_equal(E[e0:e0 + p["K"]], one.energies().cpu().numpy())
        off += a.size
        e0 += p["K"]


@pytest.mark.parametrize("iters", [0, 500])
@pytest.mark.parametrize("precision", [ssm.SSM_FP64, ssm.SSM_FP32_MIXED])
def test_full_size_tube_sampled_sites(oracle, precision, iters):
    """256x256x8, 48 images, at iteration 0 and after the workload's 500
    iterations (graph replay): fields at sampled sites of the current string
    against the direct sum."""
    w = inputs.WORKLOADS["tube_256x256x8_k48"]
    p = prob(w["nx"], w["ny"], w["nz"], w["K"], w["J"], w["d"], w["ku"], w["D"])
    s0 = inputs.build_string(w)
    if precision != ssm.SSM_FP64:
        s0 = s0.astype(np.float32).astype(np.float64)
    sm = ssm.StringMethod(p, precision)
    sm.set_options(check_every=50, graph_chunk=10)
    sm.set_string(s0)
    if iters:
        sm.iterate(iters, w["tau"])
        assert sm.check() == 0
        s0 = sm.get_string().cpu().numpy().astype(np.float64).reshape(s0.shape)
    sm.eval()
    h = sm.fields().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    N = w["nx"] * w["ny"] * w["nz"]
    tol = TOL64 if precision == ssm.SSM_FP64 else TOL32_FIELD
    for k in (0, 23, 47):
        sites = rng.choice(N, size=16, replace=False)
        sites[:4] = [0, N - 1, w["nx"] - 1, N // 2]
        ho = oracle.field_at(s0[k], p["J"], p["d"], p["ku"], p["D"], sites)
        hk = h[k].reshape(3, N)[:, sites].T
        assert rel_field(hk, ho) < tol
    del sm
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shape,precision", [
    ((1024, 1024, 1), ssm.SSM_FP64), ((1024, 1024, 1), ssm.SSM_FP32_MIXED),
    ((6, 1024, 2), ssm.SSM_FP64), ((5, 1000, 6), ssm.SSM_FP32_MIXED),
    ((1024, 7, 16), ssm.SSM_FP64), ((1000, 9, 16), ssm.SSM_FP32_MIXED),
    ((700, 700, 1), ssm.SSM_FP64), ((700, 600, 3), ssm.SSM_FP32_MIXED)])
def test_largest_shapes_sampled_sites(oracle, shape, precision):
    """The largest lattices the limits accept (1024 sites along x or y, the
    most layers the LDS allows with a 1024-point y transform, 16 layers; the
    longest 3 2^a half lengths, 768 along x and y), random spins: fields at
    sampled sites against the oracle's direct sum."""
    nx, ny, nz = shape
    K = 3
    p = prob(nx, ny, nz, K, d=0.3, ku=0.1, D=0.02)
    s0 = inputs.random_unit_spins((K, 3, nz, ny, nx), seed=nx + ny + nz)
    if precision != ssm.SSM_FP64:
        s0 = s0.astype(np.float32).astype(np.float64)
    sm = ssm.StringMethod(p, precision)
    sm.set_string(s0)
    _, h, _ = sm.eval(want_terms=False)
    h = h.cpu().numpy().astype(np.float64)
    N = nx * ny * nz
    rng = np.random.default_rng(3)
    tol = TOL64 if precision == ssm.SSM_FP64 else TOL32_FIELD
    for k in range(K):
        sites = rng.choice(N, size=12, replace=False)
        sites[:4] = [0, N - 1, nx - 1, N // 2]
        ho = oracle.field_at(s0[k], p["J"], p["d"], p["ku"], p["D"], sites)
        hk = h[k].reshape(3, N)[:, sites].T
        assert rel_field(hk, ho) < tol
    del sm
    torch.cuda.empty_cache()


def test_autograd_matches_finite_differences(oracle):
    p = prob(6, 5, 2, 3, J=1.0, d=0.3, ku=0.1, D=0.05)
    sm = ssm.StringMethod(p, ssm.SSM_FP64)
    s = torch.tensor(inputs.random_unit_spins((3, 3, 2, 5, 6), 12), device="cuda", requires_grad=True)
    th = torch.tensor([1.0, 0.3, 0.1, 0.05], dtype=torch.float64, requires_grad=True)
    E = ssm.spin_energy(s, th, sm)
    g = torch.tensor([0.3, -1.2, 0.7], dtype=torch.float64, device="cuda")
    (E * g).sum().backward()
    gs = s.grad.cpu().numpy()
    gt = th.grad.numpy()
    s_np = s.detach().cpu().numpy()
    # analytic: -h weighted; check against FD of the oracle energy on a few entries
    eps = 1e-4
    rng = np.random.default_rng(1)
    for _ in range(8):
        k = rng.integers(3)
        idx = tuple(rng.integers(n) for n in (3, 2, 5, 6))
        sp = s_np[k].copy(); sp[idx] += eps
        sm_ = s_np[k].copy(); sm_[idx] -= eps
        fd = (oracle.energy(sp, 1.0, 0.3, 0.1, 0.05) - oracle.energy(sm_, 1.0, 0.3, 0.1, 0.05)) / (2 * eps)
        assert abs(gs[k][idx] - float(g[k]) * fd) < 1e-8 * max(1.0, abs(fd))
    To = np.stack([oracle.energy_terms(si) for si in s_np])
    np.testing.assert_allclose(gt, (g.cpu().numpy()[:, None] * To).sum(0), rtol=1e-10, atol=1e-10)
