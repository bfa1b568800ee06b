"""Brute-force dense assembly of the discretised operator (oracle; test infrastructure).

No FFT, no Toeplitz structure: entry (p, i; q, j) of the 3N x 3N matrix is the
method-of-moments value of section 2.2 for the cell pair (i, j), i.e. G^E(r_i - r_j) h^3
off the diagonal and the self-cell ball integral on it.  Vector ordering matches
the field layout [3, nz, ny, nx] flattened (component-major).  Meant for grids up
to about 8^3 (1536 x 1536 complex).
"""
from __future__ import annotations

import numpy as np

from .green import green_tensor, self_term


def cell_positions(n, h, origin):
    nx, ny, nz = n
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)


def green_matrix(n, h, origin, k0, sigma0):
    """Dense G as a [3N, 3N] complex matrix."""
    r = cell_positions(n, h, origin)
    N = r.shape[0]
    Rvec = r[:, None, :] - r[None, :, :]
    diag = np.arange(N)
    Rvec[diag, diag] = (1.0, 0.0, 0.0)          # placeholder for the singular cell
    G = green_tensor(Rvec, k0, sigma0) * h ** 3  # [N, N, 3, 3]
    G[diag, diag] = self_term(h, k0, sigma0) * np.eye(3)
    return np.transpose(G, (2, 0, 3, 1)).reshape(3 * N, 3 * N)


def block_diag_tensor(T):
    """Per-cell 3x3 tensor field [3, 3, nz, ny, nx] as a sparse-in-spirit dense [3N, 3N] matrix."""
    N = T[0, 0].size
    M = np.zeros((3 * N, 3 * N), dtype=np.result_type(T.dtype, np.float64))
    idx = np.arange(N)
    for p in range(3):
        for q in range(3):
            M[p * N + idx, q * N + idx] = T[p, q].ravel()
    return M


def system_matrix(n, h, origin, k0, sigma0, dsig):
    """Dense A = I - G dsigma of eq. (8)."""
    G = green_matrix(n, h, origin, k0, sigma0)
    D = block_diag_tensor(dsig)
    return np.eye(G.shape[0]) - G @ D


def dense_solve(n, h, origin, k0, sigma0, dsig, E0):
    A = system_matrix(n, h, origin, k0, sigma0, dsig)
    return np.linalg.solve(A, E0.ravel()).reshape(E0.shape)
