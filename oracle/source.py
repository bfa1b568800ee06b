"""Background (homogeneous-medium) fields of point dipoles (oracle; test infrastructure).

Section 2.1, eqs. (1)-(2) with sigma = sigma0: the magnetic source term J^H is
not spelled out; the reading used here is J^H = i omega mu0 m delta(r - r_s)
for a magnetic dipole of moment m.  Then the background electric field is the
curl of the vector potential,
    E0 = i omega mu0 curl(m g) = i omega mu0 grad g x m
       = i omega mu0 (1 - i k0 R) exp(i k0 R) / (4 pi R^2) (m x Rhat),
and the background magnetic field is H0 = sigma0 G^E(R) m.
An electric dipole p gives E0 = G^E(R) p (the kernel of eq. 3 acting on a point current).
"""
from __future__ import annotations

import numpy as np

from .green import MU0, green_tensor


def e0_magnetic_dipole(points, pos, moment, k0, freq):
    """E0 at ``points`` [..., 3] of a magnetic dipole ``moment`` at ``pos`` -> [..., 3] complex."""
    omega = 2.0 * np.pi * freq
    Rvec = np.asarray(points, dtype=np.float64) - np.asarray(pos, dtype=np.float64)
    R = np.asarray(np.sqrt(np.sum(Rvec * Rvec, axis=-1)))
    rh = Rvec / R[..., None]
    amp = 1j * omega * MU0 * (1.0 - 1j * k0 * R) * np.exp(1j * k0 * R) / (4.0 * np.pi * R ** 2)
    m = np.asarray(moment, dtype=np.float64)
    return np.asarray(amp)[..., None] * np.cross(np.broadcast_to(m, rh.shape), rh)


def e0_electric_dipole(points, pos, moment, k0, sigma0):
    """E0 = G^E(r - r_s) p of an electric dipole ``moment`` at ``pos``."""
    Rvec = np.asarray(points, dtype=np.float64) - np.asarray(pos, dtype=np.float64)
    G = green_tensor(Rvec, k0, sigma0)
    return np.einsum("...ij,j->...i", G, np.asarray(moment, dtype=np.complex128))


def h0_magnetic_dipole(points, pos, moment, k0, sigma0):
    """H0 = sigma0 G^E(R) m of a magnetic dipole."""
    Rvec = np.asarray(points, dtype=np.float64) - np.asarray(pos, dtype=np.float64)
    G = green_tensor(Rvec, k0, sigma0)
    return sigma0 * np.einsum("...ij,j->...i", G, np.asarray(moment, dtype=np.complex128))


def background_field(n, h, origin, sources, k0, freq, sigma0):
    """E0 on cell centres, layout [3, nz, ny, nx] complex, summed over ``sources``."""
    nx, ny, nz = n
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    pts = np.stack([X, Y, Z], axis=-1)
    E = np.zeros((nz, ny, nx, 3), dtype=np.complex128)
    for pos, mom, kind in sources:
        if kind == "magnetic":
            E += e0_magnetic_dipole(pts, pos, mom, k0, freq)
        elif kind == "electric":
            E += e0_electric_dipole(pts, pos, mom, k0, sigma0)
        else:
            raise ValueError(f"unknown source kind {kind!r}")
    return np.moveaxis(E, -1, 0).copy()
