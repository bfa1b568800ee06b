"""Full-domain solves (oracle; test infrastructure).

Builds the discrete system of eq. (8) for a ``synth.Problem`` and solves it by
restarted GMRES (section 2.2), either directly in the form of eq. (8)
("conventional", the paper's choice) or in the equivalent contraction form
(see ``operator``).  Initial guess: the background field, as Alg. 1 initialises
E := E0.  The anomalous field is E - E0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import green, operator, source
from .gmres import gmres


@dataclass
class Setup:
    n: tuple
    h: float
    origin: tuple
    sigma0: float
    freq: float
    k0: complex
    Ghat: np.ndarray   # [3, 3, Lz, Ly, Lx]
    dsig: np.ndarray   # [3, 3, nz, ny, nx]
    E0: np.ndarray     # [3, nz, ny, nx]


def setup(problem, L=None):
    k0 = green.wavenumber(problem.sigma0, problem.freq)
    Ghat = green.kernel_spectrum(problem.n, problem.h, k0, problem.sigma0, L)
    dsig = operator.contrast(problem.sigma6, problem.sigma0)
    E0 = source.background_field(problem.n, problem.h, problem.origin, problem.sources,
                                 k0, problem.freq, problem.sigma0)
    return Setup(tuple(problem.n), problem.h, tuple(problem.origin), problem.sigma0,
                 problem.freq, k0, Ghat, dsig, E0)


def solve_system(Ghat, dsig, rhs, n, sigma0, form="cie", x0=None, tol=1e-6, restart=10,
                 max_its=2000):
    """Solve (I - G dsigma) x = rhs on one grid (full domain or one block)."""
    if form == "conventional":
        return gmres(lambda v: operator.apply_A(Ghat, dsig, v, n), rhs, x0, tol, restart, max_its)
    if form == "cie":
        b, a, a_inv = operator.cie_tensors(dsig, sigma0)
        s = np.sqrt(sigma0)
        y0 = None if x0 is None else operator.tensor_apply(a, x0)
        y, info = gmres(lambda v: operator.apply_C(Ghat, b, v, sigma0, n), s * rhs, y0, tol,
                        restart, max_its)
        return operator.tensor_apply(a_inv, y), info
    raise ValueError(form)


def solve_full(st: Setup, form="cie", tol=1e-6, restart=10, x0=None, max_its=5000):
    """Full-domain solve of eq. (8); returns (E, info) with info['relres'] recomputed by eq. (9)."""
    if x0 is None:
        x0 = st.E0
    E, info = solve_system(st.Ghat, st.dsig, st.E0, st.n, st.sigma0, form, x0, tol, restart,
                           max_its)
    info["relres_eq9"] = operator.relres(st.Ghat, st.dsig, E, st.E0, st.n)
    return E, info
