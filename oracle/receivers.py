"""Magnetic field at receiver points (eqs. 4 and 6); oracle, test infrastructure only.

Eq. (6) applied to eq. (5): the curl of the grad-grad term vanishes, so
    G^H(r, r') = (i omega mu0)^-1 curl G^E = curl(g I),   G^H J = grad g(r - r') x J,
with grad g(R) = (i k0 R - 1) exp(i k0 R) / (4 pi R^3) R (R = r - r').
Eq. (4) discretised like eq. (8) (collocation at cell centres, cell volume h^3):
    H(r) = H0(r) + h^3 sum_c grad g(r - r_c) x (dsigma E)_c.
Reading: a receiver exactly at a cell centre (within 1e-9 h) gets nothing from that cell, whose
kernel is odd about the receiver (its integral over the cell's equal-volume ball is zero).
Background field: magnetic dipole H0 = sigma0 G^E m (source.h0_magnetic_dipole); electric dipole
H0 = G^H p = grad g x p.
"""
from __future__ import annotations

import numpy as np

from .green import MU0  # noqa: F401  (documentation of the constant set used)
from .source import h0_magnetic_dipole


def grad_g(Rvec, k0):
    """grad g at separations Rvec [..., 3] (nonzero) -> [..., 3] complex."""
    Rvec = np.asarray(Rvec, dtype=np.float64)
    R = np.sqrt(np.sum(Rvec * Rvec, axis=-1))
    f = (1j * k0 * R - 1.0) * np.exp(1j * k0 * R) / (4.0 * np.pi * R ** 3)
    return f[..., None] * Rvec


def magnetic_green_apply(Rvec, J, k0):
    """G^H(R) J = grad g(R) x J for separations Rvec [..., 3] and currents J [..., 3]."""
    return np.cross(grad_g(Rvec, k0), np.asarray(J, dtype=np.complex128))


def h_background(points, sources, k0, sigma0):
    """H0 at points [P, 3] summed over sources [(pos, moment, kind)] -> [P, 3] complex."""
    pts = np.asarray(points, dtype=np.float64)
    H = np.zeros(pts.shape, dtype=np.complex128)
    for pos, mom, kind in sources:
        if kind == "magnetic":
            H += h0_magnetic_dipole(pts, pos, mom, k0, sigma0)
        elif kind == "electric":
            H += magnetic_green_apply(pts - np.asarray(pos, dtype=np.float64),
                                      np.broadcast_to(np.asarray(mom, dtype=np.complex128),
                                                      pts.shape), k0)
        else:
            raise ValueError(f"unknown source kind {kind!r}")
    return H


def h_anomalous(n, h, origin, dsig, E, points, k0):
    """Scattered magnetic field at points [P, 3] from the cell currents dsigma E.
    dsig: [3, 3, nz, ny, nx] real; E: [3, nz, ny, nx] complex."""
    nx, ny, nz = n
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    centres = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    J = np.einsum("pq...,q...->p...", dsig, E).reshape(3, -1).T  # [N, 3]
    out = np.zeros((len(points), 3), dtype=np.complex128)
    for k, r in enumerate(np.asarray(points, dtype=np.float64)):
        Rv = r[None, :] - centres
        R = np.sqrt(np.sum(Rv * Rv, axis=-1))
        keep = R > 1e-9 * h
        out[k] = h ** 3 * np.sum(magnetic_green_apply(Rv[keep], J[keep], k0), axis=0)
    return out


def h_total(n, h, origin, dsig, E, points, sources, k0, sigma0):
    return h_background(points, sources, k0, sigma0) + h_anomalous(n, h, origin, dsig, E, points, k0)
