"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1804_07135_amd import inputs, ssm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssm.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_list():
    assert header_functions() == sorted(ssm.ABI_SYMBOLS)


def test_binding_constants_match_the_header():
    """Every #define SSM_* of the header has the same value in the binding."""
    text = open(HEADER).read()
    defs = re.findall(r"^#define (SSM_[A-Z0-9_]+)\s+\(?(-?(?:0x[0-9a-fA-F]+|\d+))\)?", text, flags=re.M)
    assert len(defs) >= 18
    for name, val in defs:
        assert getattr(ssm, name) == int(val, 0), name


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ssm.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name


def test_version_and_kernel_names():
    assert ssm.ssm_version() >= 1
    names = [ssm.ssm_kernel_name(i) for i in range(ssm.SSM_N_KERNELS)]
    assert names[0] == "k_xfwd" and names[1] == "k_conv" and names[2] == "k_xinv"
    assert ssm.ssm_kernel_name(ssm.SSM_N_KERNELS) is None
    assert ssm.ssm_kernel_name(-1) is None


def prob(**kw):
    p = dict(nx=8, ny=8, nz=1, K=4, J=1.0, d=0.3, ku=0.1, D=0.01)
    p.update(kw)
    return p


@pytest.mark.parametrize("bad,status", [
    (dict(K=1), ssm.SSM_EINVAL),
    (dict(nx=0), ssm.SSM_EINVAL),
    (dict(nz=0), ssm.SSM_EINVAL),
    (dict(J=float("nan")), ssm.SSM_EINVAL),
    (dict(nx=2000), ssm.SSM_EUNSUPPORTED),
    (dict(nz=17), ssm.SSM_EUNSUPPORTED),
    (dict(ny=512, nz=8), ssm.SSM_EUNSUPPORTED),
    (dict(K=2000), ssm.SSM_EUNSUPPORTED),
])
def test_workspace_size_rejects(bad, status):
    with pytest.raises(ssm.SSMError) as ei:
        ssm.ssm_workspace_size([prob(**bad)], ssm.SSM_FP64)
    assert ei.value.status == status
    assert ssm.ssm_last_error(None) != ""


def half_len(n, axis="x", nz=1):
    """The documented half padded length of the x or y axis (the same rule
    for both, any layer count): the power of two >= n, or for n > 32 the
    length 3 2^a >= n (a >= 4, at most 768) when that is smaller."""
    p2 = 1 << (n - 1).bit_length()
    t = 48
    while t < n:
        t *= 2
    return t if n > 32 and t < p2 and t <= 768 else p2


def test_half_lengths():
    ns = (1, 3, 32, 33, 48, 49, 64, 65, 96, 97, 100, 129, 192, 200, 257, 300, 500, 513, 700, 769, 1024)
    want = [1, 4, 32, 48, 48, 64, 64, 96, 96, 128, 128, 192, 192, 256, 384, 384, 512, 768, 768, 1024, 1024]
    assert [half_len(n, "x") for n in ns] == want
    assert [half_len(n, "y") for n in ns] == want
    assert [half_len(n, "y", nz=12) for n in ns] == want


@pytest.mark.parametrize("precision,cap", [(ssm.SSM_FP64, 10240), (ssm.SSM_FP32_MIXED, 20480)])
@pytest.mark.parametrize("ny", [70, 100, 150, 256, 300, 700, 1024])
def test_lds_limit_is_the_documented_one(precision, cap, ny):
    """The convolution keeps its twiddles and one (y, z) plane of x-spectra
    in LDS: m_y (2 + 3 nz) complex values, at most 10240 in FP64 and 20480 in
    FP32 (160 KiB), with m_y the half padded y length; nz <= 16 regardless."""
    for nz in range(1, 17):
        my = half_len(ny, "y", nz)
        fits = my * (2 + 3 * nz) <= cap
        if fits:
            assert ssm.ssm_workspace_size([prob(ny=ny, nz=nz)], precision) > 0
        else:
            with pytest.raises(ssm.SSMError) as ei:
                ssm.ssm_workspace_size([prob(ny=ny, nz=nz)], precision)
            assert ei.value.status == ssm.SSM_EUNSUPPORTED


def test_accepted_images_fit_32_bit_byte_offsets():
    """The x kernels address one image's spins (3 N values) and its x half
    spectra ((m_x + 1) 3 nz ny complex values, m_x the power of two >= nx)
    with 32-bit byte offsets: every lattice the limits accept keeps both
    under 2^32 bytes, counted at FP64 width in either form."""
    nx = 1024
    mx = 1 << (nx - 1).bit_length()
    accepted = []
    for precision in (ssm.SSM_FP64, ssm.SSM_FP32_MIXED):
        for ny in (1, 7, 64, 100, 256, 300, 512, 640, 1000, 1024):
            for nz in range(1, 17):
                try:
                    ssm.ssm_workspace_size([prob(nx=nx, ny=ny, nz=nz)], precision)
                except ssm.SSMError:
                    continue
                accepted.append((ny, nz))
                assert 3 * nx * ny * nz * 8 < 2 ** 32
                assert (mx + 1) * 3 * nz * ny * 16 < 2 ** 32
    assert (1024, 1) in accepted and max(nz for _, nz in accepted) == 16
    with pytest.raises(ssm.SSMError):
        ssm.ssm_workspace_size([prob(nx=nx + 1)], ssm.SSM_FP32_MIXED)


def test_workspace_size_rejects_precision_and_mixed_nz():
    with pytest.raises(ssm.SSMError) as ei:
        ssm.ssm_workspace_size([prob()], 7)
    assert ei.value.status == ssm.SSM_EINVAL
    with pytest.raises(ssm.SSMError) as ei:
        ssm.ssm_workspace_size([prob(nz=2), prob(nz=8)], ssm.SSM_FP64)
    assert ei.value.status == ssm.SSM_EUNSUPPORTED
    # nz 3 and 4 share the padded z length: accepted
    assert ssm.ssm_workspace_size([prob(nz=3), prob(nz=4)], ssm.SSM_FP64) > 0


def test_workspace_sizes_scale():
    w = inputs.WORKLOADS["tube_256x256x8_k48"]
    p = dict(nx=w["nx"], ny=w["ny"], nz=w["nz"], K=w["K"], J=1, d=0.3, ku=0.1, D=0.02)
    b64 = ssm.ssm_workspace_size([p], ssm.SSM_FP64)
    b32 = ssm.ssm_workspace_size([p], ssm.SSM_FP32_MIXED)
    n = 48 * 3 * 256 * 256 * 8
    # spins, stepped spins, field, two x-spectra: about 3*8 + 2*16 bytes per value (FP64)
    assert 50 * n < b64 < 64 * n
    assert 0.45 < b32 / b64 < 0.55
    sweep = inputs.sweep_points()
    ps = [dict(nx=q["nx"], ny=q["ny"], nz=1, K=q["K"], J=q["J"], d=q["d"], ku=q["ku"], D=q["D"])
          for q in sweep]
    assert ssm.ssm_workspace_size(ps, ssm.SSM_FP32_MIXED) > 0


def test_create_rejects_null_workspace():
    lib = ssm.load()
    arr = ssm._problems([prob()])
    ctx = ctypes.c_void_p()
    st = lib.ssm_create(arr, 1, 0, None, 1 << 20, None, ctypes.byref(ctx))
    assert st == ssm.SSM_EINVAL
    assert ctx.value is None
    st = lib.ssm_create(arr, 1, 0, ctypes.c_void_p(4096 + 8), 1 << 20, None, ctypes.byref(ctx))
    assert st == ssm.SSM_EINVAL  # misaligned
    assert "aligned" in ssm.ssm_last_error(None)


def test_null_context_calls():
    lib = ssm.load()
    assert lib.ssm_destroy(None) == ssm.SSM_OK
    assert lib.ssm_iterate(None, 1, 0.1, 0.0, None) == ssm.SSM_EINVAL
    assert lib.ssm_set_string(None, None) == ssm.SSM_EINVAL
    assert lib.ssm_get_barrier(None, None) == ssm.SSM_EINVAL
