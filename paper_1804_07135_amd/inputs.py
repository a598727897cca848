"""Seeded synthetic inputs: initial strings and the benchmark workloads.

This module holds no arithmetic of the string method itself (no field, no
descent step, no reparametrisation); it only builds the initial strings the
paper describes in Sec. IV and the parameter sets of the workloads, in FP64
on the host.  Both the HIP path and the oracle are fed from here.

Initial strings (Sec. IV):
  - Bloch-point annihilation: images interpolate between the Neel skyrmion
    and the ferromagnet.  Each skyrmion spin lies in its own vertical radial
    plane, so the per-spin geodesic interpolation toward +z has the closed
    form theta_k(r) = (1 - t_k) * theta(r), t_k = k/(K-1).
  - Boundary annihilation: the skyrmion is shifted toward one edge, image by
    image, until it has left the sample; the last image is the exact
    ferromagnet.

The skyrmion profile is theta(r) = 2*atan(R/r) centred at ((nx-1)/2, (ny-1)/2),
core along -z, in-plane part pointing inward (the chirality favoured by d > 0
with the DMI sign of eq. (1)).  A "tube" repeats the profile in every layer.
Perturbation: s <- normalise(s + amp * xi), xi ~ N(0,1) i.i.d., drawn from
numpy's default_rng(seed) in C order of the array shape (K, 3, nz, ny, nx).
"""
import numpy as np


def skyrmion_angles(nx, ny, R, cx=None, cy=None):
    """Polar angle theta and azimuth phi of a Neel skyrmion on an nx x ny grid."""
    if cx is None:
        cx = (nx - 1) / 2.0
    if cy is None:
        cy = (ny - 1) / 2.0
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    rx = x - cx
    ry = y - cy
    r = np.hypot(rx, ry)
    theta = 2.0 * np.arctan2(R, r)
    phi = np.arctan2(ry, rx)
    return theta, phi


def _spins_from_angles(theta, phi, nz):
    st = np.sin(theta)
    s2 = np.stack([-st * np.cos(phi), -st * np.sin(phi), np.cos(theta)])  # [3, ny, nx]
    return np.repeat(s2[:, None, :, :], nz, axis=1)                       # [3, nz, ny, nx]


def neel_skyrmion(nx, ny, nz, R, cx=None, cy=None):
    """One image [3, nz, ny, nx]: a Neel skyrmion (tube when nz > 1)."""
    theta, phi = skyrmion_angles(nx, ny, R, cx, cy)
    return _spins_from_angles(theta, phi, nz)


def ferromagnet(nx, ny, nz, axis=2):
    s = np.zeros((3, nz, ny, nx))
    s[axis] = 1.0
    return s


def bloch_point_string(nx, ny, nz, K, R):
    """K images from the skyrmion (k=0) to the +z ferromagnet (k=K-1)."""
    theta, phi = skyrmion_angles(nx, ny, R)
    out = np.empty((K, 3, nz, ny, nx))
    for k in range(K):
        t = k / (K - 1)
        out[k] = _spins_from_angles((1.0 - t) * theta, phi, nz)
    return out


def boundary_string(nx, ny, nz, K, R):
    """K images: the skyrmion translated along +x past the edge; last = +z FM."""
    cx = (nx - 1) / 2.0
    cy = (ny - 1) / 2.0
    x_end = nx - 1 + 2.0 * R
    out = np.empty((K, 3, nz, ny, nx))
    for k in range(K):
        t = k / (K - 1)
        out[k] = neel_skyrmion(nx, ny, nz, R, cx + t * (x_end - cx), cy)
    out[K - 1] = ferromagnet(nx, ny, nz)
    return out


def perturb(s, seed, amp=1e-3):
    """normalise(s + amp * xi) with xi from default_rng(seed), C order of s."""
    s = np.asarray(s, dtype=np.float64)
    xi = np.random.default_rng(seed).standard_normal(s.shape)
    v = s + amp * xi
    n = np.sqrt((v * v).sum(axis=-4, keepdims=True))
    return v / n


def random_unit_spins(shape, seed):
    """Uniformly random unit spins, shape [..., 3, nz, ny, nx]."""
    v = np.random.default_rng(seed).standard_normal(shape)
    return v / np.sqrt((v * v).sum(axis=-4, keepdims=True))


# ---------------------------------------------------------------------------
# Workloads.  Reduced units: J is the energy unit, D = mu0 |S|^2/(4 pi a^3).
# ---------------------------------------------------------------------------
WORKLOADS = {
    "bloch_32x32x1_k10": dict(nx=32, ny=32, nz=1, K=10, J=1.0, d=0.3, ku=0.1, D=0.01,
                              R=5.0, kind="bloch", iters=200, tau=0.1, seed=1),
    "boundary_64x64x1_k20": dict(nx=64, ny=64, nz=1, K=20, J=1.0, d=0.3, ku=0.1, D=0.01,
                                 R=5.0, kind="boundary", iters=200, tau=0.1, seed=2),
    "bloch_128x128x4_k32": dict(nx=128, ny=128, nz=4, K=32, J=1.0, d=0.25, ku=0.08, D=0.02,
                                R=12.0, kind="bloch", iters=200, tau=0.1, seed=3),
    "tube_256x256x8_k48": dict(nx=256, ny=256, nz=8, K=48, J=1.0, d=0.3, ku=0.1, D=0.02,
                               R=20.0, kind="bloch", iters=500, tau=0.1, seed=5),
}


def build_string(w):
    """Initial perturbed string [K,3,nz,ny,nx] for a workload dict."""
    if w["kind"] == "bloch":
        s = bloch_point_string(w["nx"], w["ny"], w["nz"], w["K"], w["R"])
    elif w["kind"] == "boundary":
        s = boundary_string(w["nx"], w["ny"], w["nz"], w["K"], w["R"])
    else:
        raise ValueError(w["kind"])
    return perturb(s, w["seed"])


def sweep_points(n_side=8, seed=4):
    """The batched (k_u, d) sweep: n_side^2 points on k_u in [0.05, 0.2],
    d in [0.1, 0.4]; square L x L x 1 lattices, L uniform in {48..96} from
    default_rng(seed); 16 images, J = 1, D = 0.01, R = 5, Bloch-point string
    perturbed with seed 1000*seed + point index."""
    rng = np.random.default_rng(seed)
    Ls = rng.integers(48, 97, size=n_side * n_side)
    pts = []
    for i in range(n_side):
        for j in range(n_side):
            p = i * n_side + j
            ku = 0.05 + 0.15 * i / (n_side - 1)
            d = 0.1 + 0.3 * j / (n_side - 1)
            pts.append(dict(nx=int(Ls[p]), ny=int(Ls[p]), nz=1, K=16, J=1.0, d=d, ku=ku,
                            D=0.01, R=5.0, kind="bloch", tau=0.1, seed=1000 * seed + p))
    return pts


def n_sites(w):
    return w["nx"] * w["ny"] * w["nz"]
