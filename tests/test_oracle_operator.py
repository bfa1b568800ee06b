"""Pins of the oracle's FFT operator (eq. 10), system (eq. 8), residual (eq. 9) and the
contraction form, against dense brute force, dense LU and closed-form properties."""
import numpy as np
import pytest

import synth
from oracle import dense, green, operator, solve
from oracle.gmres import gmres


def _rand_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("n,L", [((8, 8, 8), None), ((6, 5, 4), None), ((5, 4, 3), (9, 8, 7)),
                                 ((4, 6, 5), (8, 16, 9))])
def test_fft_convolution_equals_dense_brute_force(n, L):
    """Eq. (10) with padding (2n, or any L >= 2n-1) reproduces the dense sum over all cell pairs."""
    p = synth.random_problem(n, seed=2)
    k0 = green.wavenumber(p.sigma0, 2e6)
    Ghat = green.kernel_spectrum(p.n, p.h, k0, p.sigma0, L)
    Gm = dense.green_matrix(p.n, p.h, p.origin, k0, p.sigma0)
    x = _rand_field((3, n[2], n[1], n[0]), 5)
    s_fft = operator.apply_green(Ghat, x, p.n).ravel()
    s_dense = Gm @ x.ravel()
    assert np.linalg.norm(s_fft - s_dense) / np.linalg.norm(s_dense) < 1e-13


def test_operator_is_complex_symmetric():
    """Reciprocity: u^T (G v) = v^T (G u) without conjugation."""
    n = (7, 6, 5)
    p = synth.random_problem(n, seed=3)
    k0 = green.wavenumber(p.sigma0, 4e5)
    Ghat = green.kernel_spectrum(p.n, p.h, k0, p.sigma0)
    u = _rand_field((3, 5, 6, 7), 1)
    v = _rand_field((3, 5, 6, 7), 2)
    a = np.sum(u * operator.apply_green(Ghat, v, n))
    b = np.sum(v * operator.apply_green(Ghat, u, n))
    assert abs(a - b) / abs(a) < 1e-13


def test_contraction_form_residual_identity_and_same_solution():
    """C = sqrt(sigma0) (I - G dsigma) a^-1: residual of the C system is sqrt(sigma0) times
    the eq. (8) residual; both forms give the same E as dense LU."""
    p = synth.random_problem((8, 8, 8), seed=4, contrast=5.0)
    st = solve.setup(p)
    b, a, a_inv = operator.cie_tensors(st.dsig, p.sigma0)
    # a a^-1 = I and b = dsigma a^-1 / (2 sqrt(sigma0)) per cell
    x = _rand_field((3, 8, 8, 8), 9)
    assert np.allclose(operator.tensor_apply(a, operator.tensor_apply(a_inv, x)), x, atol=1e-13)
    e_t = _rand_field((3, 8, 8, 8), 10)
    rC = np.sqrt(p.sigma0) * st.E0 - operator.apply_C(st.Ghat, b, e_t, p.sigma0, p.n)
    rA = st.E0 - operator.apply_A(st.Ghat, st.dsig, operator.tensor_apply(a_inv, e_t), p.n)
    assert np.linalg.norm(rC - np.sqrt(p.sigma0) * rA) / np.linalg.norm(rC) < 1e-13
    Ed = dense.dense_solve(p.n, p.h, p.origin, st.k0, p.sigma0, st.dsig, st.E0)
    for form in ("conventional", "cie"):
        E, info = solve.solve_full(st, form=form, tol=1e-12)
        assert info["converged"]
        assert np.linalg.norm(E - Ed) / np.linalg.norm(Ed) < 1e-10
        assert info["relres_eq9"] < 1e-11


def test_zero_contrast_returns_background_field():
    p = synth.random_problem((6, 6, 6), seed=5)
    p.sigma6[:] = 0.0
    p.sigma6[:3] = p.sigma0
    st = solve.setup(p)
    for form in ("conventional", "cie"):
        E, info = solve.solve_full(st, form=form, tol=1e-10)
        assert info["its"] == 0
        assert np.abs(E - st.E0).max() <= 1e-14 * np.abs(st.E0).max()


def test_born_limit_is_second_order():
    """Scaling dsigma by t: ||E(t) - E0 - t G dsigma E0|| = O(t^2)."""
    p = synth.random_problem((6, 6, 6), seed=6, contrast=3.0)
    st = solve.setup(p)
    errs = []
    for t in (1e-2, 5e-3):
        dsig = t * st.dsig / 1.0
        E = dense.dense_solve(p.n, p.h, p.origin, st.k0, p.sigma0, dsig, st.E0)
        born = st.E0 + operator.apply_green(st.Ghat, operator.tensor_apply(dsig, st.E0), p.n)
        errs.append(np.linalg.norm(E - born))
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_relres_definition_on_dense_system():
    """Eq. (9) from the FFT operator equals the dense residual."""
    p = synth.random_problem((6, 5, 4), seed=7, contrast=2.0)
    st = solve.setup(p)
    A = dense.system_matrix(p.n, p.h, p.origin, st.k0, p.sigma0, st.dsig)
    E = _rand_field(st.E0.shape, 11)
    r = st.E0.ravel() - A @ E.ravel()
    e_dense = np.linalg.norm(r) / np.linalg.norm(st.E0)
    assert abs(operator.relres(st.Ghat, st.dsig, E, st.E0, p.n) - e_dense) / e_dense < 1e-12


def test_gmres_on_known_spectra():
    """GMRES on a diagonal matrix with k distinct eigenvalues terminates in at most k steps;
    on a random well-conditioned system it matches numpy.linalg.solve."""
    rng = np.random.default_rng(12)
    lam = np.array([1.0, 2.0 + 1j, -0.5 + 0.3j, 3.0])
    d = np.repeat(lam, 25)
    b = rng.normal(size=100) + 1j * rng.normal(size=100)
    x, info = gmres(lambda v: d * v, b, tol=1e-12, restart=10)
    assert info["converged"] and info["its"] <= 4
    assert np.allclose(x, b / d, rtol=1e-10)
    M = np.eye(60) + 0.3 * (rng.normal(size=(60, 60)) + 1j * rng.normal(size=(60, 60))) / np.sqrt(60)
    b = rng.normal(size=60) + 1j * rng.normal(size=60)
    x, info = gmres(lambda v: M @ v, b, tol=1e-12, restart=10)
    assert info["converged"] and info["restarts"] >= 1
    assert np.linalg.norm(x - np.linalg.solve(M, b)) / np.linalg.norm(x) < 1e-10
    x0 = np.linalg.solve(M, b)
    x, info = gmres(lambda v: M @ v, b, x0=x0, tol=1e-10)
    assert info["its"] == 0


def test_config0_solution_has_c4v_symmetry():
    """config0 (VTI, horizontal interface, z dipole on the grid axis) is symmetric under
    90-degree rotations about z, E(R r) = R E(r), and under the vertical mirror x -> -x the
    field of an axial (magnetic) dipole flips, E(M r) = -M E(r)."""
    p = synth.config0()
    st = solve.setup(p)
    E, info = solve.solve_full(st, form="cie", tol=1e-11)
    assert info["converged"]
    Ex, Ey, Ez = E
    scale = np.abs(E).max()
    # rotation R by +90 deg about z, (x, y) -> (-y, x): rot90 over (y, x) gives E o R,
    # which must equal R E = (-Ey, Ex, Ez)
    rot = lambda A: np.rot90(A, k=1, axes=(1, 2))  # noqa: E731
    assert np.abs(rot(Ex) + Ey).max() < 1e-9 * scale
    assert np.abs(rot(Ey) - Ex).max() < 1e-9 * scale
    assert np.abs(rot(Ez) - Ez).max() < 1e-9 * scale
    # mirror x -> -x: E(M r) = -M E(r), M = diag(-1, 1, 1)
    mir = np.array([Ex[:, :, ::-1], -Ey[:, :, ::-1], -Ez[:, :, ::-1]])
    assert np.abs(mir - E).max() < 1e-9 * scale


def test_app_c_rotated_ti_tensor():
    """App. C: the rotated VTI tensor has eigenvalues {sh, sh, sv}; theta = 0 gives VTI; the
    six explicit entries of App. C match the generator term by term."""
    sh, sv = 2.0, 0.4
    for th, ph in [(0.0, 0.0), (0.3, 1.1), (1.2, -0.4), (np.pi / 3, 0.0)]:
        ax = synth.models.axis_from_angles(th, ph)
        s6 = synth.ti_tensor6(sh, sv, ax)
        S = synth.tensor6_to_3x3(s6)
        assert np.allclose(np.sort(np.linalg.eigvalsh(S)), np.sort([sh, sh, sv]))
        d = sv - sh
        app_c = [sh + d * np.sin(th) ** 2 * np.cos(ph) ** 2,
                 sh + d * np.sin(th) ** 2 * np.sin(ph) ** 2,
                 sv - d * np.sin(th) ** 2,
                 d * np.sin(th) ** 2 * np.sin(ph) * np.cos(ph),
                 d * np.sin(th) * np.cos(th) * np.cos(ph),
                 d * np.sin(th) * np.cos(th) * np.sin(ph)]
        assert np.allclose(s6, app_c, atol=1e-15)
    vti = synth.ti_tensor6(sh, sv, (0.0, 0.0, 1.0))
    assert np.allclose(vti, [sh, sh, sv, 0, 0, 0])


def test_voxel_sphere_static_field_approaches_sphere_and_is_scale_free():
    """Eq. (8) in the static limit with a uniform applied field: a sphere of conductivity sigma1 in
    sigma0 carries the uniform interior field 3 sigma0 / (sigma1 + 2 sigma0) times the applied one
    (textbook sphere in a uniform field).  A voxelised sphere approaches that value as the voxels
    shrink, and since the static problem has no length scale the discrete solution must not change
    when h does: both fail if the off-diagonal weight h^3, its sign or the kernel's static part
    (the R^-3 dipole term of eq. 5) is wrong."""
    sigma0, s1 = 0.1, 1.0
    k0 = green.wavenumber(sigma0, 1e-2)
    means = {}
    fields = {}
    for nn in (12, 16):
        for h in (0.5, 2.0):
            n = (nn, nn, nn)
            X, Y, Z = synth.cell_centres(n, h, synth.default_origin(n, h))
            inside = X ** 2 + Y ** 2 + Z ** 2 < ((nn / 2 - 1.5) * h) ** 2
            Ghat = green.kernel_spectrum(n, h, k0, sigma0)
            dsig = np.zeros((3, 3) + inside.shape)
            for p in range(3):
                dsig[p, p][inside] = s1 - sigma0
            E0 = np.zeros((3,) + inside.shape, dtype=np.complex128)
            E0[0] = 1.0
            E, info = gmres(lambda v: operator.apply_A(Ghat, dsig, v, n), E0, E0.copy(), 1e-12,
                            20, 2000)
            assert info["converged"]
            means[nn, h] = E[0][inside].real.mean()
            fields[nn, h] = E
    exact = 3 * sigma0 / (s1 + 2 * sigma0)
    for nn in (12, 16):
        # equal up to the O((k0 L)^2) dynamic correction, ~1e-6 at 10 mHz
        assert np.linalg.norm(fields[nn, 0.5] - fields[nn, 2.0]) < 1e-5 * np.linalg.norm(
            fields[nn, 0.5])
    assert abs(means[16, 0.5] - exact) < 0.05 * exact
    assert abs(means[16, 0.5] - exact) < abs(means[12, 0.5] - exact)
