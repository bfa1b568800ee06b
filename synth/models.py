"""Synthetic layered / dipping transversely-isotropic models on a regular voxel grid.

Conventions (shared by every consumer of these inputs):

* a grid is ``n = (nx, ny, nz)`` cubic cells of side ``h``; cell ``(i, j, k)``
  has its centre at ``origin + (i + 1/2, j + 1/2, k + 1/2) h``;
* grids are centred on the origin (``origin = -n h / 2`` per axis) and ``z``
  points down (depth);
* conductivity is stored as six real components per cell in the order
  ``xx, yy, zz, xy, xz, yz``, array shape ``[6, nz, ny, nx]`` (x fastest);
* a transmitter is a point dipole ``(pos[3], moment[3], kind)`` with ``kind``
  ``"magnetic"`` (default) or ``"electric"``;
* a sub-domain partition is the list of z cell indices ``0 = z_0 < ... < z_M = nz``.

The transversely-isotropic tensor in a tilted frame is App. C's rotated VTI
tensor, written as ``sigma_h I + (sigma_v - sigma_h) n n^T`` with the symmetry
axis ``n = (sin t cos p, sin t sin p, cos t)``; expanding ``n n^T`` gives the
six entries of App. C term by term.

Every random draw uses ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SIGMA0_DEFAULT = 0.1  # S/m, background used by every workload here


@dataclass
class Problem:
    """One forward problem: grid, medium, tensors, transmitters, partition."""

    name: str
    n: tuple            # (nx, ny, nz)
    h: float            # cell size (m)
    origin: tuple       # corner of cell (0, 0, 0) (m)
    sigma0: float       # background conductivity (S/m)
    freq: float         # Hz
    sigma6: np.ndarray  # [6, nz, ny, nx] float64
    sources: list = field(default_factory=list)  # [(pos, moment, kind)]
    z_bounds: tuple = ()  # sub-domain partition along z

    @property
    def ncell(self) -> int:
        nx, ny, nz = self.n
        return nx * ny * nz


def default_origin(n, h):
    return tuple(-0.5 * ni * h for ni in n)


def cell_centres(n, h, origin):
    """Return X, Y, Z arrays of shape [nz, ny, nx] with the cell-centre coordinates."""
    nx, ny, nz = n
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def axis_from_angles(theta, phi):
    """Symmetry axis of a tilted TI medium: polar angle theta, azimuth phi (radians)."""
    return np.array([math.sin(theta) * math.cos(phi),
                     math.sin(theta) * math.sin(phi),
                     math.cos(theta)])


def ti_tensor6(sigma_h, sigma_v, axis):
    """Six components (xx, yy, zz, xy, xz, yz) of sigma_h I + (sigma_v - sigma_h) a a^T.

    ``sigma_h`` and ``sigma_v`` may be arrays (broadcast together); ``axis`` is a unit 3-vector.
    """
    sh = np.asarray(sigma_h, dtype=np.float64)
    sv = np.asarray(sigma_v, dtype=np.float64)
    a = np.asarray(axis, dtype=np.float64)
    d = sv - sh
    return np.stack([
        sh + d * a[0] * a[0],
        sh + d * a[1] * a[1],
        sh + d * a[2] * a[2],
        d * a[0] * a[1],
        d * a[0] * a[2],
        d * a[1] * a[2],
    ])


def tensor6_to_3x3(sigma6):
    """[6, ...] -> [3, 3, ...] symmetric tensor field."""
    s = np.asarray(sigma6)
    xx, yy, zz, xy, xz, yz = s
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def _layer_index(s, interfaces):
    """Index of the layer that contains signed distance s (interfaces sorted ascending)."""
    return np.searchsorted(np.asarray(interfaces, dtype=np.float64), s, side="right")


def _layered_sigma6(n, h, origin, normal, interfaces, sig_h, sig_v):
    """Cells classified by the signed distance of their centre along ``normal``; no averaging."""
    X, Y, Z = cell_centres(n, h, origin)
    s = normal[0] * X + normal[1] * Y + normal[2] * Z
    lay = _layer_index(s, interfaces)
    sh = np.asarray(sig_h)[lay]
    sv = np.asarray(sig_v)[lay]
    return ti_tensor6(sh, sv, normal)


def _log_uniform(rng, lo, hi, size=None):
    return 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=size)


def _sorted_offsets(rng, count, lo, hi, min_gap):
    while True:
        d = np.sort(rng.uniform(lo, hi, size=count))
        if count < 2 or np.all(np.diff(d) >= min_gap):
            return d


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def config0():
    """16^3 cells of 0.5 m; upper half background, lower half VTI (1, 0.2) S/m; 100 kHz;
    unit z magnetic dipole 1 m above the grid centre; no partition."""
    n = (16, 16, 16)
    h = 0.5
    origin = default_origin(n, h)
    _, _, Z = cell_centres(n, h, origin)
    sig0 = SIGMA0_DEFAULT
    lower = Z > 0.0
    sh = np.where(lower, 1.0, sig0)
    sv = np.where(lower, 0.2, sig0)
    sigma6 = ti_tensor6(sh, sv, (0.0, 0.0, 1.0))
    src = [((0.0, 0.0, -1.0), (0.0, 0.0, 1.0), "magnetic")]
    return Problem("config0_16cube_two_layer_vti", n, h, origin, sig0, 1.0e5, sigma6, src, (0, 16))


def _three_layer_dipping(n, h, seed, freq, z_bounds, name):
    rng = np.random.Generator(np.random.PCG64(seed))
    normal = axis_from_angles(math.radians(30.0), 0.0)
    d = _sorted_offsets(rng, 2, -4.0, 4.0, 2.0)
    sig_h = _log_uniform(rng, 0.01, 10.0, size=3)
    sig_v = sig_h / 5.0
    origin = default_origin(n, h)
    sigma6 = _layered_sigma6(n, h, origin, normal, d, sig_h, sig_v)
    src = [((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), "magnetic")]
    return Problem(name, n, h, origin, SIGMA0_DEFAULT, freq, sigma6, src, tuple(z_bounds))


def config1(seed=101, n=(64, 64, 64), h=0.25):
    """64^3 cells of 0.25 m, three tilted-TI layers dipping 30 deg (sigma_h/sigma_v = 5,
    sigma_h log-uniform in [0.01, 10] S/m), 2 MHz, z dipole at the centre, two z slabs."""
    nz = n[2]
    return _three_layer_dipping(n, h, seed, 2.0e6, (0, nz // 2, nz),
                                f"config1_{n[0]}x{n[1]}x{n[2]}_3layer_dip30_seed{seed}")


def config3(seed=303, n=(128, 128, 256), h=0.25):
    """128x128x256 cells of 0.25 m, six tilted-TI layers dipping 20 deg, principal values
    in [0.1, 10] S/m, 2 MHz, z dipole at the centre, four z slabs of 64.  Other n and h give
    the same layers (interface offsets in metres) on another grid, in four equal z slabs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    normal = axis_from_angles(math.radians(20.0), 0.0)
    d = _sorted_offsets(rng, 5, -24.0, 24.0, 3.0)
    sig_h = _log_uniform(rng, 0.1, 10.0, size=6)
    lam = rng.choice(np.array([1.0, 2.0, 5.0]), size=6)
    sig_v = np.maximum(sig_h / lam, 0.1)
    origin = default_origin(n, h)
    sigma6 = _layered_sigma6(n, h, origin, normal, d, sig_h, sig_v)
    src = [((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), "magnetic")]
    nz = n[2]
    return Problem(f"config3_{n[0]}x{n[1]}x{n[2]}_h{h}_6layer_dip20_seed{seed}", n, h, origin,
                   SIGMA0_DEFAULT, 2.0e6, sigma6, src, (0, nz // 4, nz // 2, 3 * nz // 4, nz))


CONFIG2_SHAPES = ((32, 32, 32), (48, 48, 64), (64, 64, 96))


def config2(seed=202, positions=64, freqs=(4.0e5, 2.0e6)):
    """Logging run: ``positions`` tool positions along a straight trajectory 60 deg from
    vertical (0.5 m apart) through four horizontal TI layers, each position solved at
    every frequency in ``freqs`` on a tool-centred local grid whose z axis follows the
    trajectory.  Returns the list of problems (position-major)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    depths = np.array([3.0, 8.0, 13.0]) + rng.uniform(-1.0, 1.0, size=3)
    sig_h = _log_uniform(rng, 0.1, 10.0, size=4)
    lam = rng.uniform(1.0, 5.0, size=4)
    sig_v = sig_h / lam
    theta = math.radians(60.0)
    t = np.array([math.sin(theta), 0.0, math.cos(theta)])       # tool z' (world)
    ex = np.array([-math.cos(theta), 0.0, math.sin(theta)])     # tool x' (world)
    ey = np.cross(t, ex)                                        # right-handed frame
    # the world vertical seen from the tool frame: (ex.z, ey.z, t.z) = F7 axis with phi = 0
    axis_tool = np.array([ex[2], ey[2], t[2]])
    shape_idx = rng.integers(0, len(CONFIG2_SHAPES), size=positions)
    h = 0.25
    out = []
    for k in range(positions):
        p = k * 0.5 * t
        n = CONFIG2_SHAPES[shape_idx[k]]
        origin = default_origin(n, h)
        X, Y, Z = cell_centres(n, h, origin)
        depth = p[2] + X * ex[2] + Y * ey[2] + Z * t[2]
        lay = _layer_index(depth, depths)
        sigma6 = ti_tensor6(sig_h[lay], sig_v[lay], axis_tool)
        nb = 3 if n[2] == 96 else 2
        zb = tuple(int(round(i * n[2] / nb)) for i in range(nb + 1))
        for f in freqs:
            out.append(Problem(f"config2_pos{k:02d}_{n[0]}x{n[1]}x{n[2]}_{int(f / 1e3)}kHz",
                               n, h, origin, SIGMA0_DEFAULT, f, sigma6,
                               [((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), "magnetic")], zb))
    return out


def _random_block_sample(seed, n=(32, 32, 32), h=0.25):
    rng = np.random.Generator(np.random.PCG64(seed))
    nlay = int(rng.integers(2, 5))
    dip = math.radians(rng.uniform(0.0, 60.0))
    az = rng.uniform(0.0, 2.0 * math.pi)
    normal = axis_from_angles(dip, az)
    half = 0.5 * n[2] * h
    d = np.sort(rng.uniform(-half, half, size=nlay - 1))
    sig_h = _log_uniform(rng, 0.01, 10.0, size=nlay)
    lam = rng.uniform(1.0, 5.0, size=nlay)
    sig_v = sig_h / lam
    freq = float(rng.choice(np.array([1.0e5, 4.0e5, 2.0e6])))
    origin = default_origin(n, h)
    sigma6 = _layered_sigma6(n, h, origin, normal, d, sig_h, sig_v)
    ext = np.array([ni * h for ni in n]) * 0.5
    while True:   # uniform in the 2 m shell outside the block faces
        pos = rng.uniform(-(ext + 2.0), ext + 2.0)
        if np.any(np.abs(pos) > ext):
            break
    m = rng.normal(size=3)
    m /= np.linalg.norm(m)
    src = [(tuple(pos), tuple(m), "magnetic")]
    return Problem(f"config4_train_seed{seed}", n, h, origin, SIGMA0_DEFAULT, freq,
                   sigma6, src, (0, n[2]))


def config4_train(start=40000, count=2000):
    """Training blocks for the learned initial guess (one seed per sample)."""
    for s in range(start, start + count):
        yield _random_block_sample(s)


def config4_eval(start=50000, count=16):
    """Held-out 64^3 evaluation models in the style of the three-layer dipping workload."""
    for s in range(start, start + count):
        yield config1(seed=s)


def example1(n=128, h=0.25):
    """Two isolated isotropic 0.01 S/m anomalies of 30 x 30 x 7.5 m in the 0.1 S/m background,
    10 m apart along z (about one background skin depth at 24 kHz), symmetric about a
    transmitter at the origin oriented along x (the isolated sub-domains example, sec. 3.1; its
    figure is not reproduced, so the anomalies are placed symmetrically about the transmitter).
    The partition separates the two anomalies and the three zero-contrast slabs."""
    nn = (n, n, n)
    origin = default_origin(nn, h)
    sig = np.zeros((6, n, n, n))
    sig[:3] = SIGMA0_DEFAULT
    ext = int(round(30.0 / h))     # 120 cells at 0.25 m
    thick = int(round(7.5 / h))    # 30 cells
    gap = int(round(10.0 / h))     # 40 cells
    x0 = (n - ext) // 2
    z_a0 = (n - gap) // 2 - thick
    z_b0 = (n + gap) // 2
    for z0 in (z_a0, z_b0):
        sig[:3, z0:z0 + thick, x0:x0 + ext, x0:x0 + ext] = 0.01
    src = [((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), "magnetic")]
    zb = (0, z_a0, z_a0 + thick, z_b0, z_b0 + thick, n)
    return Problem(f"example1_{n}cubed_two_isolated_anomalies", nn, h, origin, SIGMA0_DEFAULT,
                   2.4e4, sig, src, zb)


def random_problem(n, h=0.25, seed=0, freq=1.0e5, sigma0=SIGMA0_DEFAULT, contrast=1.0,
                   z_bounds=None, src_offset=(0.3, -0.2, -1.1)):
    """Small random anisotropic model: each cell a random SPD tensor around
    ``sigma0 (1 + contrast u)``, for parity tests at arbitrary shapes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = n
    A = rng.normal(size=(nz, ny, nx, 3, 3)) * 0.3
    S = np.einsum("...ij,...kj->...ik", A, A)
    base = sigma0 * (1.0 + contrast * rng.uniform(0.0, 1.0, size=(nz, ny, nx)))
    S = S * sigma0 * contrast + base[..., None, None] * np.eye(3)
    sigma6 = np.stack([S[..., 0, 0], S[..., 1, 1], S[..., 2, 2],
                       S[..., 0, 1], S[..., 0, 2], S[..., 1, 2]])
    origin = default_origin(n, h)
    zc = origin[2] - 1.0 if src_offset is None else src_offset[2]
    src = [((src_offset[0], src_offset[1], zc), (0.2, -0.3, 0.93), "magnetic")]
    zb = tuple(z_bounds) if z_bounds is not None else (0, nz)
    return Problem(f"random_{nx}x{ny}x{nz}_seed{seed}", tuple(n), h, origin, sigma0, freq,
                   sigma6, src, zb)
