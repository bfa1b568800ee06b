"""GPU parity of the learned-initial-guess network (hand-written BF16 MFMA kernels) against the
CPU reference network: the GEMM operand layout, the forward pass, parameter gradients, the Adam
step and a short training run.

Tolerances.  The reference run with ``quant=True`` rounds to bfloat16 at the same points as the
GPU, so the GPU differs from it only through float32 accumulation order (relative 1e-6 per sum)
and the bf16 roundings that this order flips (a flip moves a value by one bf16 step, 2^-8
relative, and is rare).  Measured gaps are far below the 2e-3 (forward) and 1e-2 (gradients)
bars used here.  The exact float64 network is a looser sanity bound: bf16 stores each value with
a 2^-9 relative error, the forward output is within 3e-2 of it, and the whole parameter
gradient, rounded once per layer on its way down, within 0.1 (single tensors, bias sums with
heavy cancellation above all, can be further off, so they are held to the quantised run only).
"""
import numpy as np
import pytest

from oracle import cnn
from tests.gpu_common import banner, dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _bf16_dev(torch, a):
    return dev(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).contiguous()


@pytest.mark.parametrize("a_trans,b_trans", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K,splits", [(16, 16, 16, 1), (77, 45, 100, 1), (77, 45, 100, 3),
                                          (130, 70, 300, 5), (1, 1, 1, 1), (64, 64, 32, 1)])
def test_gemm_operand_layout(torch, a_trans, b_trans, M, N, K, splits):
    from paper_2306_17537_amd import ie
    banner(f"nn gemm M={M} N={N} K={K} at={a_trans} bt={b_trans} splits={splits}")
    rng = np.random.default_rng(M * 7 + N + K)
    A = cnn.bf16(rng.normal(size=(M, K)))
    B = cnn.bf16(rng.normal(size=(K, N)))
    Ad = _bf16_dev(torch, A.T.copy() if a_trans else A)
    Bd = _bf16_dev(torch, B.T.copy() if b_trans else B)
    Cd = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda:0")
    ie.ie_nn_gemm(Ad, Bd, Cd, M, N, K, a_trans, b_trans, splits)
    ref = A @ B
    scale = np.abs(A) @ np.abs(B)
    err = np.abs(host(Cd).astype(np.float64) - ref)
    assert np.all(np.isfinite(host(Cd)))
    assert np.all(err <= 1e-6 * K * scale + 1e-30), float(np.max(err / (scale + 1e-30)))


CFGS = [
    (dict(in_ch=3, out_ch=2, base=4, levels=3), 2, (4, 8, 12)),
    (dict(in_ch=5, out_ch=3, base=3, levels=1), 1, (3, 5, 7)),
    (dict(in_ch=14, out_ch=6, base=8, levels=4), 1, (8, 8, 16)),
]


def _net(ie, cfg, seed):
    return ie.ie_nn_create(cfg["in_ch"], cfg["out_ch"], cfg["base"], cfg["levels"], seed)


@pytest.mark.parametrize("ci", range(len(CFGS)))
def test_forward_matches_reference(torch, ci):
    from paper_2306_17537_amd import ie
    cfg, nb, (Z, Y, X) = CFGS[ci]
    banner(f"nn forward cfg={cfg} nb={nb} grid={(Z, Y, X)}")
    net = _net(ie, cfg, 11 + ci)
    try:
        flat = ie.ie_nn_get_params(net).astype(np.float64)
        assert flat.size == cnn.num_params(cnn.layer_specs(**cfg))
        # biases start at zero; give them values so the bias path is exercised
        rng = np.random.default_rng(ci)
        flat = flat + 0.05 * rng.normal(size=flat.size)
        ie.ie_nn_set_params(net, flat)
        flat = ie.ie_nn_get_params(net).astype(np.float64)  # float32 master copy
        x = cnn.bf16(rng.normal(size=(nb, Z, Y, X, cfg["in_ch"])))
        y = torch.full((nb, Z, Y, X, cfg["out_ch"]), float("nan"), dtype=torch.float32,
                       device="cuda:0")
        ie.ie_nn_forward(net, _bf16_dev(torch, x), y)
        got = host(y).astype(np.float64)
        ref_q = cnn.forward(x, flat, **cfg, quant=True)
        ref = cnn.forward(x, flat, **cfg)
        banner(f"  rel vs quantised {rel(got, ref_q):.2e}, vs exact {rel(got, ref):.2e}")
        assert rel(got, ref_q) < 2e-3
        assert rel(got, ref) < 3e-2
    finally:
        ie.ie_nn_destroy(net)


@pytest.mark.parametrize("ci", range(len(CFGS)))
def test_gradients_match_reference(torch, ci):
    from paper_2306_17537_amd import ie
    cfg, nb, (Z, Y, X) = CFGS[ci]
    banner(f"nn backward cfg={cfg} nb={nb} grid={(Z, Y, X)}")
    net = _net(ie, cfg, 21 + ci)
    try:
        rng = np.random.default_rng(100 + ci)
        flat = ie.ie_nn_get_params(net).astype(np.float64) + 0.05 * rng.normal(
            size=ie.ie_nn_num_params(net))
        ie.ie_nn_set_params(net, flat)
        flat = ie.ie_nn_get_params(net).astype(np.float64)
        x = cnn.bf16(rng.normal(size=(nb, Z, Y, X, cfg["in_ch"])))
        gy = rng.normal(size=(nb, Z, Y, X, cfg["out_ch"])).astype(np.float32)
        y = torch.empty((nb, Z, Y, X, cfg["out_ch"]), dtype=torch.float32, device="cuda:0")
        ie.ie_nn_backward(net, _bf16_dev(torch, x), dev(gy), y)
        torch.cuda.synchronize()
        g = ie.ie_nn_get_params(net, which=1).astype(np.float64)
        ref_q = cnn.backward(x, flat, gy.astype(np.float64), **cfg, quant=True)
        ref = cnn.backward(x, flat, gy.astype(np.float64), **cfg)
        specs = cnn.layer_specs(**cfg)
        o = 0
        worst = 0.0
        for name, c_in, c_out, taps, _ in specs:
            for part, size in (("W", taps * c_in * c_out), ("b", c_out)):
                sl = slice(o, o + size)
                e = rel(g[sl], ref_q[sl])
                worst = max(worst, e)
                assert e < 1e-2, (name, part, e)
                o += size
        banner(f"  worst per-tensor gradient rel vs quantised {worst:.2e}, "
               f"whole gradient vs exact {rel(g, ref):.2e}")
        assert o == g.size
        assert rel(g, ref) < 0.1
    finally:
        ie.ie_nn_destroy(net)


def test_first_adam_step_and_loss(torch):
    from paper_2306_17537_amd import ie
    cfg, nb, (Z, Y, X) = CFGS[0]
    banner("nn first Adam step")
    net = _net(ie, cfg, 31)
    try:
        rng = np.random.default_rng(7)
        flat = ie.ie_nn_get_params(net).astype(np.float64)
        x = cnn.bf16(rng.normal(size=(nb, Z, Y, X, cfg["in_ch"])))
        t = rng.normal(size=(nb, Z, Y, X, cfg["out_ch"])).astype(np.float32)
        lr = 1e-3
        loss = ie.ie_nn_train_step(net, _bf16_dev(torch, x), dev(t), lr)
        yq = cnn.forward(x, flat, **cfg, quant=True)
        ref_loss = np.mean((yq - t) ** 2)
        assert abs(loss - ref_loss) <= 2e-3 * ref_loss, (loss, ref_loss)
        # first Adam step from zero moments: p -= lr g / (|g| + eps), i.e. about lr sign(g)
        g = cnn.backward(x, flat, 2.0 * (yq - t) / yq.size, **cfg, quant=True)
        new = ie.ie_nn_get_params(net).astype(np.float64)
        d = new - flat
        assert np.all(np.abs(d) <= lr * (1 + 1e-3) + 1e-7)
        big = np.abs(g) > 1e-2 * np.max(np.abs(g))
        assert np.all(np.abs(d[big] + lr * np.sign(g[big])) <= 2e-2 * lr + 1e-7)
    finally:
        ie.ie_nn_destroy(net)


def test_training_reduces_loss(torch):
    """A student network learns a fixed teacher network's map on fixed inputs."""
    from paper_2306_17537_amd import ie
    cfg = dict(in_ch=4, out_ch=2, base=8, levels=3)
    banner("nn training run")
    teacher = _net(ie, cfg, 41)
    student = _net(ie, cfg, 42)
    try:
        rng = np.random.default_rng(8)
        x = _bf16_dev(torch, rng.normal(size=(4, 8, 8, 8, 4)))
        t = torch.empty((4, 8, 8, 8, 2), dtype=torch.float32, device="cuda:0")
        ie.ie_nn_forward(teacher, x, t)
        losses = [ie.ie_nn_train_step(student, x, t, 2e-3) for _ in range(150)]
        banner(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
        assert np.all(np.isfinite(losses))
        assert losses[-1] < 0.1 * losses[0]
    finally:
        ie.ie_nn_destroy(teacher)
        ie.ie_nn_destroy(student)
