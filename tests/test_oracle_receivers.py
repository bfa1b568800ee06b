"""Pins of the receiver magnetic field (eqs. 4 and 6): the magnetic kernel against Faraday's law
applied by finite differences to the electric kernel of eq. (5), the background field of both
source kinds, and the zero-contrast limit."""
import numpy as np

import synth
from oracle import green, operator, receivers, source
from oracle.green import MU0


def _curl(f, r, d=1e-5):
    """Central-difference curl of a vector field f: R^3 -> C^3 at r."""
    J = np.zeros((3, 3), dtype=np.complex128)  # J[i, j] = d f_i / d x_j
    for j in range(3):
        e = np.zeros(3)
        e[j] = d
        J[:, j] = (f(r + e) - f(r - e)) / (2 * d)
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])


def test_magnetic_kernel_is_curl_of_electric_kernel():
    sigma0, freq = 0.1, 2.0e6
    k0 = green.wavenumber(sigma0, freq)
    omega = 2 * np.pi * freq
    rp = np.array([0.3, -0.2, 0.1])
    Jc = np.array([0.4 - 0.2j, -1.0 + 0.5j, 0.7j])
    E = lambda r: green.green_tensor((r - rp)[None], k0, sigma0)[0] @ Jc  # noqa: E731
    for r in (np.array([1.1, 0.4, -0.7]), np.array([-0.5, 2.0, 1.5]), np.array([0.0, 0.0, 3.0])):
        H_fd = _curl(E, r) / (1j * omega * MU0)
        H = receivers.magnetic_green_apply((r - rp)[None], Jc[None], k0)[0]
        assert np.allclose(H, H_fd, rtol=1e-6, atol=1e-9 * np.abs(H).max())


def test_background_fields_obey_faraday():
    sigma0, freq = 0.1, 4.0e5
    k0 = green.wavenumber(sigma0, freq)
    omega = 2 * np.pi * freq
    pos, m = (0.1, 0.2, -0.3), (0.3, -0.5, 0.8)
    r = np.array([0.9, -0.6, 1.2])
    for kind in ("magnetic", "electric"):
        if kind == "magnetic":
            E = lambda q: source.e0_magnetic_dipole(q[None], pos, m, k0, freq)[0]  # noqa: E731
        else:
            E = lambda q: source.e0_electric_dipole(q[None], pos, m, k0, sigma0)[0]  # noqa: E731
        # away from the source curl E0 = i omega mu0 H0 (eq. 1 with J^H = 0 there)
        H_fd = _curl(E, r) / (1j * omega * MU0)
        H = receivers.h_background(r[None], [(pos, m, kind)], k0, sigma0)[0]
        assert np.allclose(H, H_fd, rtol=1e-6, atol=1e-9 * np.abs(H).max())


def test_zero_contrast_gives_background_and_cell_centre_receivers_skip_their_cell():
    p = synth.random_problem((4, 3, 5), seed=1, freq=1e5, contrast=0.0)
    k0 = green.wavenumber(p.sigma0, p.freq)
    dsig = operator.contrast(p.sigma6, p.sigma0)
    assert np.all(dsig == 0)
    E = np.ones((3, 5, 3, 4), dtype=np.complex128)
    pts = np.array([[0.0, 0.0, 2.0], [0.3, 0.1, -1.0]])
    src = [((0.1, 0.0, 0.0), (0.0, 0.0, 1.0), "magnetic")]
    H = receivers.h_total(p.n, p.h, p.origin, dsig, E, pts, src, k0, p.sigma0)
    assert np.array_equal(H, receivers.h_background(pts, src, k0, p.sigma0))
    # a receiver on a cell centre: identical to the sum over the other cells
    p2 = synth.random_problem((3, 3, 3), seed=2, freq=1e5, contrast=2.0)
    d2 = operator.contrast(p2.sigma6, p2.sigma0)
    E2 = np.random.default_rng(0).normal(size=(3, 3, 3, 3)) + 0j
    c = np.array([p2.origin[0] + 1.5 * p2.h, p2.origin[1] + 1.5 * p2.h, p2.origin[2] + 1.5 * p2.h])
    d_hole = d2.copy()
    d_hole[:, :, 1, 1, 1] = 0
    a = receivers.h_anomalous(p2.n, p2.h, p2.origin, d2, E2, c[None], k0)
    b = receivers.h_anomalous(p2.n, p2.h, p2.origin, d_hole, E2, c[None], k0)
    assert np.allclose(a, b, rtol=1e-14, atol=0)


def test_scattered_magnetic_field_is_curl_of_scattered_electric_field():
    """Eq. (1) away from the cells: the field of the discretised cell currents J = dsigma E obeys
    curl E^a = i omega mu0 H^a.  E^a at an off-grid point is written here as a plain sum of the
    electric kernel of eq. (5) with the operator's cell weight h^3 (checked first against the FFT
    operator of eq. 10 at a cell centre, whose own cell is the self term); its finite-difference
    curl must equal the oracle's H^a of eq. (4).  Fails if h^3, the current dsigma E, the kernel's
    sign or the sum over cells is wrong in either."""
    p = synth.random_problem((4, 3, 5), seed=3, freq=4e5, contrast=2.0)
    k0 = green.wavenumber(p.sigma0, p.freq)
    omega = 2 * np.pi * p.freq
    dsig = operator.contrast(p.sigma6, p.sigma0)
    rng = np.random.default_rng(4)
    E = rng.normal(size=(3, 5, 3, 4)) + 1j * rng.normal(size=(3, 5, 3, 4))
    J = operator.tensor_apply(dsig, E)
    X, Y, Z = synth.cell_centres(p.n, p.h, p.origin)
    centres = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    Jc = J.reshape(3, -1).T

    def e_scat(r, skip=None):
        out = np.zeros(3, dtype=np.complex128)
        for c in range(len(centres)):
            if c != skip:
                out += green.green_tensor((r - centres[c])[None], k0, p.sigma0)[0] @ Jc[c] * p.h ** 3
        return out

    S = operator.apply_green(green.kernel_spectrum(p.n, p.h, k0, p.sigma0), J, p.n)
    c = 2 * 12 + 1 * 4 + 2  # cell (2, 1, 2)
    expect = S.reshape(3, -1)[:, c] - green.self_term(p.h, k0, p.sigma0) * Jc[c]
    assert np.allclose(e_scat(centres[c], skip=c), expect, rtol=1e-12, atol=0)
    pts = np.array([[0.05, 0.02, 0.1], [0.9, -0.6, 1.7], [-0.3, 0.4, -2.0]])
    for r in pts:
        H_fd = _curl(e_scat, r, d=1e-6) / (1j * omega * MU0)
        H = receivers.h_anomalous(p.n, p.h, p.origin, dsig, E, r[None], k0)[0]
        assert np.allclose(H, H_fd, rtol=1e-6, atol=1e-9 * np.abs(H).max())
