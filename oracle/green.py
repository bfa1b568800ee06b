"""Whole-space electric Green's tensor and its voxel discretisation (oracle; test infrastructure).

Follows section 2.1, eqs. (5) and (7), and section 2.2 (method of moments).

* Diffusive regime (section 2.1): conductivity is real, mu = mu0 and the time
  factor is such that the scalar Green's function decays as exp(i k0 R) with
  Im k0 > 0, where k0 = sqrt(i omega mu0 sigma0) on the principal branch.
* Eq. (5): G^E = (i omega mu0 I + grad grad / sigma0) g with g = exp(i k0 R)/(4 pi R).
  Expanding grad grad g for a radial function gives, for R != 0,
      G^E(R) = exp(i k0 R) / (4 pi sigma0 R^3)
               * [ (k0^2 R^2 + i k0 R - 1) I + (3 - 3 i k0 R - k0^2 R^2) Rhat Rhat^T ].
* Section 2.2 discretisation (reading: midpoint rule for the non-singular
  part, sphere of equal volume for the singular self cell):
      off-diagonal   Gd(i, j) = G^E(r_i - r_j) h^3,
      self cell      Gd(i, i) = I * integral of G^E over a ball of radius a,
                     a = (3 h^3 / (4 pi))^(1/3)
                   = I * [2 (1 - i k0 a) exp(i k0 a) - 3] / (3 sigma0).
  The ball integral splits into i omega mu0 * int g dV = [(1 - i k0 a) e^{i k0 a} - 1]/sigma0
  and (1/sigma0) int grad grad g dV = (1/3) I (i k0 a - 1) e^{i k0 a} / sigma0 (divergence
  theorem on the distribution grad grad g, which carries the -delta/3 term).
* Eq. (10) and the text after it: the discrete convolution is evaluated by FFT on a
  grid padded to twice the cell count per axis; the kernel value for offset d sits at
  index d mod 2n, and the unused index n is zero.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

MU0 = 4.0e-7 * np.pi  # H/m, section 2.1 sets mu = mu0


def wavenumber(sigma0: float, freq: float) -> complex:
    """k0 = sqrt(i omega mu0 sigma0), principal branch so Im k0 > 0 (eq. 7)."""
    omega = 2.0 * np.pi * freq
    return complex(np.sqrt(1j * omega * MU0 * sigma0))


def scalar_green(R, k0):
    """g(R) = exp(i k0 R) / (4 pi R) (eq. 7)."""
    R = np.asarray(R, dtype=np.float64)
    return np.exp(1j * k0 * R) / (4.0 * np.pi * R)


def green_tensor(Rvec, k0, sigma0):
    """G^E(R) of eq. (5) for separation vectors ``Rvec`` [..., 3] (all nonzero) -> [..., 3, 3]."""
    Rvec = np.asarray(Rvec, dtype=np.float64)
    R = np.asarray(np.sqrt(np.sum(Rvec * Rvec, axis=-1)))
    rh = Rvec / R[..., None]
    ikR = np.asarray(1j * k0 * R)
    pref = np.asarray(np.exp(ikR) / (4.0 * np.pi * sigma0 * R ** 3))
    kR2 = np.asarray((k0 * R) ** 2)
    a = kR2 + ikR - 1.0
    c = 3.0 - 3.0 * ikR - kR2
    eye = np.eye(3)
    return pref[..., None, None] * (a[..., None, None] * eye
                                    + c[..., None, None] * rh[..., :, None] * rh[..., None, :])


def self_term(h, k0, sigma0):
    """Diagonal value of the discretised operator: ball integral of G^E (section 2.2)."""
    a = (3.0 * h ** 3 / (4.0 * np.pi)) ** (1.0 / 3.0)
    ika = 1j * k0 * a
    return (2.0 * (1.0 - ika) * np.exp(ika) - 3.0) / (3.0 * sigma0)


def offset_kernel(n, h, k0, sigma0):
    """Discretised operator as a function of the cell offset d = i - j.

    Returns K[3, 3, 2nz-1, 2ny-1, 2nx-1] with K[..., dz + nz-1, dy + ny-1, dx + nx-1] = Gd(d).
    """
    nx, ny, nz = n
    dx = np.arange(-(nx - 1), nx)
    dy = np.arange(-(ny - 1), ny)
    dz = np.arange(-(nz - 1), nz)
    DZ, DY, DX = np.meshgrid(dz, dy, dx, indexing="ij")
    Rvec = np.stack([DX, DY, DZ], axis=-1).astype(np.float64) * h
    zero = (DX == 0) & (DY == 0) & (DZ == 0)
    Rsafe = Rvec.copy()
    Rsafe[zero] = (1.0, 0.0, 0.0)  # placeholder, overwritten below
    G = green_tensor(Rsafe, k0, sigma0) * h ** 3
    G[zero] = self_term(h, k0, sigma0) * np.eye(3)
    return np.moveaxis(G, (-2, -1), (0, 1))


def kernel_spectrum(n, h, k0, sigma0, L=None):
    """FFT of the zero-padded kernel (eq. 10): Ghat[3, 3, Lz, Ly, Lx], L = 2n unless given.

    Any L >= 2n - 1 per axis gives the same linear convolution.
    """
    nx, ny, nz = n
    if L is None:
        L = (2 * nx, 2 * ny, 2 * nz)
    Lx, Ly, Lz = L
    assert Lx >= 2 * nx - 1 and Ly >= 2 * ny - 1 and Lz >= 2 * nz - 1
    K = offset_kernel(n, h, k0, sigma0)
    P = np.zeros((3, 3, Lz, Ly, Lx), dtype=np.complex128)
    iz = np.arange(-(nz - 1), nz) % Lz
    iy = np.arange(-(ny - 1), ny) % Ly
    ix = np.arange(-(nx - 1), nx) % Lx
    P[:, :, iz[:, None, None], iy[None, :, None], ix[None, None, :]] = K
    return scipy.fft.fftn(P, axes=(2, 3, 4))
