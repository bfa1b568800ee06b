"""Domain-decomposition outer iteration, Alg. 1 (oracle; test infrastructure).

Section 2.3: the grid is split into M non-overlapping rectangular sub-domains
(here z slabs, eq. 11).  Eq. (13) gives, per sub-domain i,
    E(i) = E(i,0) + sum_j G(ij) dsigma(j) E(j),
which is the block system of eqs. (14)-(16).  With the splitting A = L + U + D
(eqs. 17-18):

* block Gauss-Seidel (eqs. 19-22): sub-domains in ascending order, each solving
  (I - G(ii) dsigma(i)) E(i)^{k+1} = E(i,0) + sum_{j<i} G(ij) dsigma(j) E(j)^{k+1}
                                            + sum_{j>i} G(ij) dsigma(j) E(j)^k;
* block Jacobi (eqs. 23-24): every coupling term from sweep k (j != i).

Each block system is solved by restarted GMRES from the previous outer iterate
(Alg. 1 and the paragraph before it).  Inner tolerance: fixed (1e-6 in section 3.2)
or adaptive, e/10 with e the full-domain relative residual of eq. (9) (Alg. 1).
Readings where Alg. 1 is garbled: e is recomputed after every sweep, the Jacobi sum
excludes j = i (eq. 24), and E at k = 0 is the background field.

The coupling term is evaluated the plainest way: one full-domain convolution of
dsigma E with the target block's own source zeroed, restricted to the target
block.  Block self operators use the block's own padded FFT grid (2 n_block per
axis), as the text after eq. (16) notes that rectangular blocks keep the FFT.
A block with zero contrast has A_ii = I, so its update is E(i) = b_i with no
inner iterations (sub-domains without anomaly are omitted from the work, section 2.3).
"""
from __future__ import annotations

import numpy as np

from . import green, operator
from .solve import Setup, solve_system


def _zmask(n, z0, z1):
    nx, ny, nz = n
    m = np.zeros((nz, ny, nx), dtype=bool)
    m[z0:z1] = True
    return m


def coupling(st: Setup, E, z0, z1):
    """sum_{j != i} G(ij) dsigma(j) E(j) on block i = [z0, z1): full-domain convolution,
    source zeroed on block i, result restricted to block i."""
    m = _zmask(st.n, z0, z1)
    J = operator.tensor_apply(st.dsig, E)
    S = operator.apply_green(st.Ghat, J, st.n, src_mask=~m)
    return S[:, z0:z1]


def dd_solve(st: Setup, z_bounds, scheme="gs", adaptive=True, tol=1e-6, inner_tol_fixed=1e-6,
             form="conventional", restart=10, max_sweeps=100, inner_max_its=5000, E_init=None,
             anomalous_only=False):
    """Alg. 1.  Returns (E, info) with per-sweep full residuals, the inner tolerance each sweep
    used and per-block iteration counts.  ``anomalous_only``: e over the cells with contrast only
    (the isolated sub-domains example, section 3.1)."""
    nx, ny, nz = st.n
    zb = list(z_bounds)
    blocks = list(zip(zb[:-1], zb[1:]))
    ghat_cache = {}

    def block_ghat(nzb):
        if nzb not in ghat_cache:
            ghat_cache[nzb] = green.kernel_spectrum((nx, ny, nzb), st.h, st.k0, st.sigma0)
        return ghat_cache[nzb]

    E = st.E0.copy() if E_init is None else np.array(E_init, dtype=np.complex128)
    e = operator.relres(st.Ghat, st.dsig, E, st.E0, st.n, anomalous_only)
    info = dict(relres=[e], block_its=[], inner_tol=[], sweeps=0, total_its=0,
                converged=e <= tol)
    while e > tol and info["sweeps"] < max_sweeps:
        E_old = E.copy()
        its_sweep = []
        inner_tol = e / 10.0 if adaptive else inner_tol_fixed
        info["inner_tol"].append(inner_tol)
        for (z0, z1) in blocks:
            src = E if scheme == "gs" else E_old
            rhs = st.E0[:, z0:z1] + coupling(st, src, z0, z1)
            dsig_i = st.dsig[:, :, z0:z1]
            if not np.any(dsig_i):
                E[:, z0:z1] = rhs
                its_sweep.append(0)
                continue
            nb = (nx, ny, z1 - z0)
            Ei, inf = solve_system(block_ghat(z1 - z0), dsig_i, rhs, nb, st.sigma0, form,
                                   x0=E_old[:, z0:z1], tol=inner_tol, restart=restart,
                                   max_its=inner_max_its)
            E[:, z0:z1] = Ei
            its_sweep.append(inf["its"])
        info["sweeps"] += 1
        info["block_its"].append(its_sweep)
        info["total_its"] += sum(its_sweep)
        e = operator.relres(st.Ghat, st.dsig, E, st.E0, st.n, anomalous_only)
        info["relres"].append(e)
    info["converged"] = e <= tol
    return E, info


def dd_sweep_from_zero(st: Setup, z_bounds, v, scheme="gs", inner_tol=1e-2, form="conventional",
                       restart=10, inner_max_its=5000, ghat_cache=None):
    """One sweep of Alg. 1 applied to A z = v from z = 0: the block Gauss-Seidel (eqs. 19-22) or
    Jacobi (eqs. 23-24) preconditioner.  Returns (z, inner iterations)."""
    nx, ny, nz = st.n
    zb = list(z_bounds)
    cache = {} if ghat_cache is None else ghat_cache
    z = np.zeros_like(np.asarray(v, dtype=np.complex128))
    its = 0
    for (z0, z1) in zip(zb[:-1], zb[1:]):
        rhs = v[:, z0:z1] + (coupling(st, z, z0, z1) if scheme == "gs" else 0.0)
        dsig_i = st.dsig[:, :, z0:z1]
        if not np.any(dsig_i):
            z[:, z0:z1] = rhs
            continue
        nzb = z1 - z0
        if nzb not in cache:
            cache[nzb] = green.kernel_spectrum((nx, ny, nzb), st.h, st.k0, st.sigma0)
        zi, inf = solve_system(cache[nzb], dsig_i, rhs, (nx, ny, nzb), st.sigma0, form,
                               x0=None, tol=inner_tol, restart=restart, max_its=inner_max_its)
        z[:, z0:z1] = zi
        its += inf["its"]
    return z, its


def fgmres_dd(st: Setup, z_bounds, scheme="gs", tol=1e-6, inner_tol=1e-2, form="conventional",
              restart=10, max_its=200, inner_max_its=5000):
    """The Krylov outer iteration in place of the stationary sweeps (the improvement proposed in
    the conclusions): flexible GMRES on the full-domain eq. (8) from E = 0, right-preconditioned
    by one sweep of Alg. 1 with inner solves to `inner_tol`.  Returns (E, info) with the outer
    GMRES info plus the total inner iterations."""
    from .gmres import fgmres
    cache = {}
    inner = [0]

    def precond(v):
        z, its = dd_sweep_from_zero(st, z_bounds, v, scheme, inner_tol, form, restart,
                                    inner_max_its, cache)
        inner[0] += its
        return z

    E, info = fgmres(lambda x: operator.apply_A(st.Ghat, st.dsig, x, st.n), precond, st.E0,
                     None, tol, restart, max_its)
    info["inner_its"] = inner[0]
    info["relres"] = operator.relres(st.Ghat, st.dsig, E, st.E0, st.n)
    return E, info
