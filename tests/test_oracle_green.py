"""Pins of the oracle's Green's tensor, its discretisation and the background field.

Each check compares the oracle with something other than its own formula:
finite differences of eqs. (5) and (7), numerical quadrature of the self-cell
ball integral, the magnetostatic limit, and the textbook field inside a small
sphere.
"""
import numpy as np
import pytest
import scipy.integrate

from oracle import green, source

SIG0 = 0.1
FREQ = 2.0e6


def _fd_hessian(f, r, d):
    H = np.zeros((3, 3), dtype=np.complex128)
    E = np.eye(3) * d
    for i in range(3):
        for j in range(3):
            H[i, j] = (f(r + E[i] + E[j]) - f(r + E[i] - E[j])
                       - f(r - E[i] + E[j]) + f(r - E[i] - E[j])) / (4 * d * d)
    return H


def _g_at(k0):
    return lambda r: complex(green.scalar_green(np.linalg.norm(r), k0))


@pytest.mark.parametrize("freq", [1.0e3, 1.0e5, 2.0e6])
def test_green_tensor_equals_fd_of_eq5(freq):
    """G^E = (i w mu0 I + grad grad / sigma0) g, with grad grad g by central differences of g."""
    k0 = green.wavenumber(SIG0, freq)
    w = 2 * np.pi * freq
    rng = np.random.default_rng(3)
    for _ in range(6):
        r = rng.normal(size=3)
        r *= rng.uniform(0.3, 3.0) / np.linalg.norm(r)
        d = 1e-4 * np.linalg.norm(r)
        Hs = _fd_hessian(_g_at(k0), r, d)
        G_fd = 1j * w * green.MU0 * complex(green.scalar_green(np.linalg.norm(r), k0)) * np.eye(3) \
            + Hs / SIG0
        G = green.green_tensor(r, k0, SIG0)
        assert np.linalg.norm(G - G_fd) / np.linalg.norm(G) < 2e-6


def test_scalar_green_solves_helmholtz_and_decays():
    """g of eq. (7) satisfies lap g + k0^2 g = 0 off the source, and decays (Im k0 > 0)."""
    k0 = green.wavenumber(SIG0, FREQ)
    assert k0.imag > 0 and k0.real > 0
    f = _g_at(k0)
    r = np.array([0.7, -0.4, 1.1])
    H = _fd_hessian(f, r, 1e-4)
    lap = np.trace(H)
    assert abs(lap + k0 ** 2 * f(r)) / abs(k0 ** 2 * f(r)) < 1e-5
    assert abs(f(10 * r)) < abs(f(r)) / 10


def test_green_tensor_symmetry_parity_trace():
    k0 = green.wavenumber(SIG0, FREQ)
    rng = np.random.default_rng(4)
    R = rng.normal(size=(20, 3))
    G = green.green_tensor(R, k0, SIG0)
    Gm = green.green_tensor(-R, k0, SIG0)
    assert np.allclose(G, np.swapaxes(G, -1, -2), rtol=0, atol=1e-14 * np.abs(G).max())
    assert np.allclose(G, Gm, rtol=1e-14, atol=0)
    r = np.linalg.norm(R, axis=-1)
    tr = np.trace(G, axis1=-2, axis2=-1)
    expect = 2 * k0 ** 2 * green.scalar_green(r, k0) / SIG0
    assert np.allclose(tr, expect, rtol=1e-12)


def test_static_limit_is_magnetostatic_dipole():
    """H0 = sigma0 G^E m tends to (3 Rhat (Rhat.m) - m) / (4 pi R^3) as omega -> 0."""
    k0 = green.wavenumber(SIG0, 1e-6)
    m = np.array([0.3, -0.5, 0.8])
    for R in ([1.0, 0.0, 0.0], [0.3, 0.4, -1.2], [-2.0, 1.0, 0.5]):
        R = np.array(R)
        H = source.h0_magnetic_dipole(R, np.zeros(3), m, k0, SIG0)
        rh = R / np.linalg.norm(R)
        Hs = (3 * rh * rh.dot(m) - m) / (4 * np.pi * np.linalg.norm(R) ** 3)
        assert np.allclose(H, Hs, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("freq,h", [(1.0e5, 0.5), (2.0e6, 0.25), (2.0e6, 1.0)])
def test_self_term_equals_ball_quadrature(freq, h):
    """Self-cell value = ball integral of G^E by quadrature: i w mu0 int g dV by radial
    quadrature, plus (1/sigma0) int grad grad g dV as the flux of grad g through the sphere
    (divergence theorem), with grad g taken by finite differences on a spherical grid."""
    k0 = green.wavenumber(SIG0, freq)
    w = 2 * np.pi * freq
    a = (3 * h ** 3 / (4 * np.pi)) ** (1 / 3)
    re = scipy.integrate.quad(lambda r: (r * np.exp(1j * k0 * r)).real, 0, a, epsabs=1e-14)[0]
    im = scipy.integrate.quad(lambda r: (r * np.exp(1j * k0 * r)).imag, 0, a, epsabs=1e-14)[0]
    vol_part = 1j * w * green.MU0 * (re + 1j * im)   # 4 pi r^2 g = r e^{ikr}
    # flux of d_j g through the sphere: Gauss-Legendre in cos(theta), uniform in phi
    ct, wt = np.polynomial.legendre.leggauss(24)
    ph = np.linspace(0, 2 * np.pi, 48, endpoint=False)
    g = _g_at(k0)
    d = 1e-5 * a
    flux = np.zeros((3, 3), dtype=np.complex128)
    for c, wc in zip(ct, wt):
        s = np.sqrt(1 - c * c)
        for p in ph:
            nvec = np.array([s * np.cos(p), s * np.sin(p), c])
            x = a * nvec
            grad = np.array([(g(x + d * e) - g(x - d * e)) / (2 * d) for e in np.eye(3)])
            flux += np.outer(nvec, grad) * wc * (2 * np.pi / len(ph)) * a * a
    G_ball = vol_part * np.eye(3) + flux / SIG0
    expect = green.self_term(h, k0, SIG0) * np.eye(3)
    assert np.linalg.norm(G_ball - expect) / np.linalg.norm(expect) < 1e-6


def test_single_cell_static_field_is_sphere_field():
    """One anomalous cell at omega -> 0: E = (I - Gself dsigma)^-1 E0 -> 3 sigma0/(sigma1 + 2 sigma0) E0,
    the textbook uniform field inside a conducting sphere."""
    k0 = green.wavenumber(SIG0, 1e-3)
    gs = green.self_term(0.5, k0, SIG0)
    for s1 in (0.01, 0.3, 10.0):
        factor = 1.0 / (1.0 - gs * (s1 - SIG0))
        assert abs(factor - 3 * SIG0 / (s1 + 2 * SIG0)) < 1e-6


def _fd_curl(F, r, d):
    J = np.zeros((3, 3), dtype=np.complex128)
    for j, e in enumerate(np.eye(3)):
        J[:, j] = (F(r + d * e) - F(r - d * e)) / (2 * d)
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])


@pytest.mark.parametrize("freq", [1.0e5, 2.0e6])
def test_background_field_of_magnetic_dipole(freq):
    """E0 = i w mu0 curl(m g) (finite-difference curl), and curl E0 = i w mu0 H0 off the source,
    which ties E0 and H0 = sigma0 G^E m together through eq. (1)."""
    k0 = green.wavenumber(SIG0, freq)
    w = 2 * np.pi * freq
    m = np.array([0.2, -0.7, 0.5])
    pos = np.array([0.1, 0.2, -0.3])
    g = _g_at(k0)
    A = lambda r: m * g(r - pos)  # noqa: E731
    E = lambda r: source.e0_magnetic_dipole(r, pos, m, k0, freq)  # noqa: E731
    rng = np.random.default_rng(7)
    for _ in range(4):
        r = pos + rng.normal(size=3)
        d = 1e-5
        E_fd = 1j * w * green.MU0 * _fd_curl(A, r, d)
        assert np.linalg.norm(E(r) - E_fd) / np.linalg.norm(E_fd) < 1e-6
        H = source.h0_magnetic_dipole(r, pos, m, k0, SIG0)
        curlE = _fd_curl(E, r, d)
        assert np.linalg.norm(curlE - 1j * w * green.MU0 * H) / np.linalg.norm(curlE) < 1e-5


def test_electric_dipole_field_satisfies_vector_helmholtz():
    """E0 = G^E p solves curl curl E - k0^2 E = 0 away from the source."""
    k0 = green.wavenumber(SIG0, FREQ)
    p = np.array([0.0, 1.0, 0.3])
    E = lambda r: source.e0_electric_dipole(r, np.zeros(3), p, k0, SIG0)  # noqa: E731
    r = np.array([0.8, -0.5, 0.6])
    d = 1e-3
    cc = _fd_curl(lambda q: _fd_curl(E, q, d), r, d)
    assert np.linalg.norm(cc - k0 ** 2 * E(r)) / np.linalg.norm(k0 ** 2 * E(r)) < 1e-4
