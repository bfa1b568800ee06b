"""The discretised integral operator and its FFT evaluation (oracle; test infrastructure).

* Eq. (8): (I - G dsigma) E = E0, with dsigma = sigma - sigma0 I (section 2.1).
* Eq. (10): each tensor component of the convolution is evaluated as
  IFFT(FFT[G_pq] * FFT[(dsigma E)_q]) on a grid zero-padded to twice the cell
  count per axis (text after eq. 10), then cropped back to the cells.
* Eq. (9): relative residual e = ||E0 - (I - G dsigma) E|| / ||E0|| (2-norm over
  all 3N entries).
* Contraction form (introduction and end of section 2.3, not used in the paper's
  runs): with b = dsigma (2 sigma0 I + dsigma)^-1 and a = (2 sigma0 I + dsigma)/(2 sqrt(sigma0))
  per cell, eq. (8) is equivalent to
      C e~ = sqrt(sigma0) E0,   C = (I - b) - 2 sigma0 G b,   E = a^-1 e~,
  and C = sqrt(sigma0) (I - G dsigma) a^-1, so the relative residual of the C system
  equals eq. (9) exactly.

Layouts: fields [3, nz, ny, nx] complex; per-cell tensors [3, 3, nz, ny, nx] real.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from synth import tensor6_to_3x3


def contrast(sigma6, sigma0):
    """dsigma = sigma - sigma0 I as [3, 3, nz, ny, nx]."""
    S = tensor6_to_3x3(sigma6).astype(np.float64)
    for p in range(3):
        S[p, p] = S[p, p] - sigma0
    return S


def _cellwise(T):
    """[3, 3, ...] -> [..., 3, 3] for per-cell linear algebra."""
    return np.moveaxis(T, (0, 1), (-2, -1))


def _uncellwise(T):
    return np.moveaxis(T, (-2, -1), (0, 1))


def cie_tensors(dsig, sigma0):
    """Per-cell b = dsigma (2 sigma0 I + dsigma)^-1 and a^-1 = 2 sqrt(sigma0) (2 sigma0 I + dsigma)^-1."""
    D = _cellwise(dsig)
    M = D + 2.0 * sigma0 * np.eye(3)
    Minv = np.linalg.inv(M)
    b = D @ Minv
    a_inv = 2.0 * np.sqrt(sigma0) * Minv
    a = M / (2.0 * np.sqrt(sigma0))
    return _uncellwise(b), _uncellwise(a), _uncellwise(a_inv)


def tensor_apply(T, x):
    """(T x)_p = sum_q T_pq x_q per cell."""
    return np.einsum("pq...,q...->p...", T, x)


def apply_green(Ghat, J, n, src_mask=None, out_mask=None):
    """S = G J by eq. (10): pad J to the FFT grid, transform, multiply by Ghat, invert, crop.

    ``src_mask``/``out_mask`` are optional boolean [nz, ny, nx] arrays: the source is zeroed
    outside ``src_mask`` and the result outside ``out_mask``.
    """
    nx, ny, nz = n
    Lz, Ly, Lx = Ghat.shape[2:]
    if src_mask is not None:
        J = J * src_mask[None]
    P = np.zeros((3, Lz, Ly, Lx), dtype=np.complex128)
    P[:, :nz, :ny, :nx] = J
    Jh = scipy.fft.fftn(P, axes=(1, 2, 3))
    Sh = np.einsum("pq...,q...->p...", Ghat, Jh)
    S = scipy.fft.ifftn(Sh, axes=(1, 2, 3))[:, :nz, :ny, :nx]
    if out_mask is not None:
        S = S * out_mask[None]
    return S


def apply_A(Ghat, dsig, x, n):
    """(I - G dsigma) x, eq. (8)."""
    return x - apply_green(Ghat, tensor_apply(dsig, x), n)


def apply_C(Ghat, b, x, sigma0, n):
    """(I - b) x - 2 sigma0 G (b x): contraction form of the same operator."""
    bx = tensor_apply(b, x)
    return x - bx - 2.0 * sigma0 * apply_green(Ghat, bx, n)


def anomalous_cells(dsig):
    """Cells whose contrast tensor is not zero ([nz, ny, nx] bool)."""
    return np.any(dsig.reshape(9, *dsig.shape[2:]) != 0, axis=0)


def relres(Ghat, dsig, E, E0, n, anomalous_only=False):
    """Eq. (9); with ``anomalous_only`` both norms run over the cells with contrast only, the
    residual the isolated sub-domains example computes (section 3.1)."""
    r = E0 - apply_A(Ghat, dsig, E, n)
    if anomalous_only:
        m = anomalous_cells(dsig)[None]
        r, E0 = r * m, E0 * m
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(E0.ravel()))
