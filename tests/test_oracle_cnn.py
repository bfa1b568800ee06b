"""Pins of the CPU reference network: convolution against scipy's N-d correlation, gradients
against central finite differences, pooling / upsampling adjointness."""
import numpy as np
import scipy.signal

from oracle import cnn


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 6, 3))
    W = rng.normal(size=(27, 3, 2))
    b = rng.normal(size=2)
    y = cnn.conv(x, W, b)
    K = W.reshape(3, 3, 3, 3, 2)  # (dz, dy, dx, ci, co)
    for n in range(2):
        for co in range(2):
            ref = b[co] + sum(scipy.signal.correlate(x[n, ..., ci], K[..., ci, co], mode="same")
                              for ci in range(3))
            assert np.allclose(y[n, ..., co], ref, atol=1e-12)


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 3, 4, 3, 2))
    W = rng.normal(size=(27, 2, 3))
    b = rng.normal(size=3)
    gy = rng.normal(size=(1, 3, 4, 3, 3))
    gx, gW, gb = cnn.conv_backward(x, W, gy)
    f = lambda xx, WW, bb: np.sum(gy * cnn.conv(xx, WW, bb))  # noqa: E731
    eps = 1e-6
    for idx in [(0, 1, 2, 0, 1), (0, 0, 0, 2, 0), (0, 2, 3, 1, 1)]:
        d = np.zeros_like(x)
        d[idx] = eps
        assert abs((f(x + d, W, b) - f(x - d, W, b)) / (2 * eps) - gx[idx]) < 1e-7
    for idx in [(0, 0, 0), (13, 1, 2), (26, 1, 1)]:
        d = np.zeros_like(W)
        d[idx] = eps
        assert abs((f(x, W + d, b) - f(x, W - d, b)) / (2 * eps) - gW[idx]) < 1e-7
    d = np.zeros_like(b)
    d[1] = eps
    assert abs((f(x, W, b + d) - f(x, W, b - d)) / (2 * eps) - gb[1]) < 1e-7


def test_pool_and_upsample_are_adjoint_up_to_factor():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 4, 4, 6, 2))
    g = rng.normal(size=(1, 2, 2, 3, 2))
    assert np.isclose(np.sum(cnn.pool(x) * g), np.sum(x * cnn.pool_backward(g)))
    u = rng.normal(size=(1, 2, 2, 3, 2))
    gu = rng.normal(size=(1, 4, 4, 6, 2))
    assert np.isclose(np.sum(cnn.upsample(u) * gu), np.sum(u * cnn.upsample_backward(gu)))


def test_network_parameter_gradient_matches_finite_differences():
    cfg = dict(in_ch=3, out_ch=2, base=2, levels=3)
    rng = np.random.default_rng(3)
    flat = cnn.init_params(**cfg, seed=7) + 0.05 * rng.normal(size=cnn.num_params(
        cnn.layer_specs(**cfg)))
    x = rng.normal(size=(1, 4, 4, 8, 3))
    gy = rng.normal(size=(1, 4, 4, 8, 2))
    g = cnn.backward(x, flat, gy, **cfg)
    assert g.shape == flat.shape
    f = lambda p: np.sum(gy * cnn.forward(x, p, **cfg))  # noqa: E731
    eps = 1e-6
    for i in rng.choice(flat.size, size=25, replace=False):
        d = np.zeros_like(flat)
        d[i] = eps
        fd = (f(flat + d) - f(flat - d)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_bf16_rounding_matches_torch_and_ties_to_even():
    import torch
    rng = np.random.default_rng(4)
    a = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-20, 20, size=1000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(a), ref)
    # ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 -> even mantissa (1); 1 + 3 * 2^-8 -> up
    assert cnn.bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert cnn.bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6


def test_quantised_network_stays_close_to_exact():
    cfg = dict(in_ch=3, out_ch=2, base=4, levels=3)
    rng = np.random.default_rng(5)
    flat = cnn.init_params(**cfg, seed=9)
    x = cnn.bf16(rng.normal(size=(1, 4, 8, 8, 3)))
    y = cnn.forward(x, flat, **cfg)
    yq = cnn.forward(x, flat, **cfg, quant=True)
    err = np.linalg.norm(yq - y) / np.linalg.norm(y)
    assert 1e-5 < err < 3e-2  # rounding happened, and only at the bf16 level (2^-9 per rounding)
