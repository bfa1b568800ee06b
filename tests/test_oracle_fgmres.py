"""Pins of the Krylov outer iteration over the DD sweep: flexible GMRES reduces to GMRES with the
identity preconditioner, converges in one step with the exact inverse, and with one Alg. 1
sweep as preconditioner reaches the dense solution in fewer outer steps than the stationary
sweeps need."""
import numpy as np

import synth
from oracle import dd, dense, gmres, operator, solve


def _small(seed=4):
    rng = np.random.default_rng(seed)
    A = np.eye(30) + 0.3 * (rng.normal(size=(30, 30)) + 1j * rng.normal(size=(30, 30))) / 6
    b = rng.normal(size=30) + 1j * rng.normal(size=30)
    return A, b


def test_fgmres_with_identity_is_gmres():
    A, b = _small()
    x1, i1 = gmres.gmres(lambda v: A @ v, b, tol=1e-12, restart=7, max_its=200)
    x2, i2 = gmres.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-12, restart=7, max_its=200)
    assert i1["its"] == i2["its"]
    assert np.allclose(x1, x2, rtol=0, atol=1e-12)
    assert np.allclose(A @ x2, b, atol=1e-10)


def test_fgmres_with_exact_inverse_takes_one_step():
    A, b = _small(5)
    Ainv = np.linalg.inv(A)
    x, info = gmres.fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-12, restart=5)
    assert info["its"] == 1
    assert np.allclose(A @ x, b, atol=1e-10)


def test_fgmres_dd_reaches_dense_solution_faster_than_sweeps():
    p = synth.random_problem((8, 8, 8), seed=9, freq=2.0e6, contrast=3.0, z_bounds=(0, 4, 8))
    st = solve.setup(p)
    ref = dense.dense_solve(p.n, p.h, p.origin, st.k0, p.sigma0, st.dsig, st.E0)
    for scheme in ("gs", "jacobi"):
        E, info = dd.fgmres_dd(st, p.z_bounds, scheme, tol=1e-10, inner_tol=1e-3)
        _, sw = dd.dd_solve(st, p.z_bounds, scheme, adaptive=False, tol=1e-10,
                            inner_tol_fixed=1e-12, max_sweeps=200)
        assert info["relres"] <= 1e-10
        assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-8
        assert info["its"] < sw["sweeps"], (scheme, info["its"], sw["sweeps"])
