"""GPU parity of the magnetic field at receivers (eqs. 4 and 6) against the oracle, on ragged
grids with receivers inside, outside and on a cell centre, both transmitter kinds, and on the
64^3 workload with the stored oracle field (the induction-log response |H_z| at 7, 15 and 30 m
from the transmitter, the spacings of the paper's logging example)."""
import os

import numpy as np
import pytest

import synth
from oracle import green, operator, receivers, source
from tests.gpu_common import banner, context, dev

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _rx_points(p, rng):
    nx, ny, nz = p.n
    lo = np.array(p.origin)
    hi = lo + p.h * np.array([nx, ny, nz])
    inside = lo + rng.uniform(0.1, 0.9, size=(3, 3)) * (hi - lo)
    outside = hi + rng.uniform(0.5, 3.0, size=(2, 3))
    centre = lo + p.h * (np.array([nx // 2, ny // 2, nz // 2]) + 0.5)
    return np.vstack([inside, outside, centre[None]])


@pytest.mark.parametrize("n", [(5, 7, 3), (16, 12, 9), (1, 1, 1), (24, 20, 33)])
@pytest.mark.parametrize("kind", ["magnetic", "electric"])
def test_receivers_match_oracle(torch, n, kind):
    from paper_2306_17537_amd import ie
    banner(f"receivers n={n} kind={kind}")
    p = synth.random_problem(n, seed=sum(n), freq=4.0e5, contrast=3.0)
    src = [(s[0], s[1], kind) for s in p.sources]
    rng = np.random.default_rng(sum(n))
    rx = _rx_points(p, rng)
    shape = (3, n[2], n[1], n[0])
    E = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    ctx, _ = context(p)
    try:
        H, Ha = ie.ie_receivers(ctx, dev(p.sigma6), src, dev(E), rx)
    finally:
        ie.ie_ctx_destroy(ctx)
    k0 = green.wavenumber(p.sigma0, p.freq)
    dsig = operator.contrast(p.sigma6, p.sigma0)
    ref_a = receivers.h_anomalous(p.n, p.h, p.origin, dsig, E, rx, k0)
    ref = receivers.h_background(rx, src, k0, p.sigma0) + ref_a
    assert np.allclose(Ha, ref_a, rtol=1e-11, atol=1e-13 * np.abs(ref_a).max())
    assert np.allclose(H, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_induction_log_response_on_the_64_cubed_workload(torch):
    from paper_2306_17537_amd import ie
    p = synth.config1()
    gold = np.load(os.path.join(ROOT, "tests", "golden", "config1_Ea.npz"))["Ea"].astype(np.complex128)
    k0 = green.wavenumber(p.sigma0, p.freq)
    E = source.background_field(p.n, p.h, p.origin, p.sources, k0, p.freq, p.sigma0) + gold
    rx = np.array([[0.0, 0.0, 7.0], [0.0, 0.0, 15.0], [0.0, 0.0, 30.0]])
    ctx, _ = context(p)
    try:
        H, Ha = ie.ie_receivers(ctx, dev(p.sigma6), p.sources, dev(E), rx)
    finally:
        ie.ie_ctx_destroy(ctx)
    dsig = operator.contrast(p.sigma6, p.sigma0)
    ref_a = receivers.h_anomalous(p.n, p.h, p.origin, dsig, E, rx, k0)
    ref = receivers.h_background(rx, p.sources, k0, p.sigma0) + ref_a
    for q in range(3):
        banner(f"spacing {rx[q, 2]:.0f} m: |Hz| = {abs(H[q, 2]):.4e} A/m (background "
               f"{abs(H[q, 2] - Ha[q, 2]):.4e}); error vs oracle {abs(H[q, 2] - ref[q, 2]):.2e}")
    # the scattered field nearly cancels the background here, so the error is measured against
    # the size of the terms summed (float64 sums in different orders), per receiver
    scale = np.abs(ref_a).max(axis=1, keepdims=True)
    assert np.all(np.abs(Ha - ref_a) <= 1e-11 * scale)
    assert np.all(np.abs(H - ref) <= 1e-11 * scale)


def test_receivers_reject_bad_input(torch):
    from paper_2306_17537_amd import ie
    p = synth.random_problem((4, 4, 4), seed=3)
    E = np.zeros((3, 4, 4, 4), dtype=np.complex128)
    ctx, _ = context(p)
    try:
        with pytest.raises(ie.IEError, match="on source"):
            ie.ie_receivers(ctx, dev(p.sigma6), p.sources, dev(E), [p.sources[0][0]])
        with pytest.raises(ie.IEError, match="nrx"):
            ie.ie_receivers(ctx, dev(p.sigma6), p.sources, dev(E), np.zeros((0, 3)))
    finally:
        ie.ie_ctx_destroy(ctx)
