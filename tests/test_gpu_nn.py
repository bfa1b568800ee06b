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


# ----------------------------------------------------------------------------------------
# solver features, targets and the residual judge
# ----------------------------------------------------------------------------------------
def _rand_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def test_features_and_target_match_reference(torch):
    """Features and targets against their definitions; a global phase of b must not change the
    features (checked by a second call with b e^{0.7 i})."""
    import synth
    from oracle import green, operator
    from paper_2306_17537_amd import ie
    from tests.gpu_common import context, field_shape
    p = synth.random_problem((6, 5, 4), seed=3, freq=4.0e5, contrast=20.0)
    banner("nn features / target")
    ctx, _ = context(p)
    try:
        nx, ny, nz = p.n
        b = _rand_field(field_shape(p), 1)
        E = _rand_field(field_shape(p), 2)
        xd = torch.empty((nz, ny, nx, 14), dtype=torch.bfloat16, device="cuda:0")
        yd = torch.empty((nz, ny, nx, 6), dtype=torch.float32, device="cuda:0")
        rms = ie.ie_nn_features(ctx, dev(p.sigma6), dev(b), xd)
        ie.ie_nn_target(ctx, dev(b), dev(E), yd)
        ref_rms = np.linalg.norm(b) / np.sqrt(b.size)
        assert abs(rms - ref_rms) <= 1e-12 * ref_rms
        rot = np.exp(-0.5j * np.angle(np.sum(b * b)))  # global phase fixed by sum b.b
        bt, _, _ = operator.cie_tensors(operator.contrast(p.sigma6, p.sigma0), p.sigma0)
        k0h = green.wavenumber(p.sigma0, p.freq) * p.h
        ref = np.zeros((nz, ny, nx, 14))
        for c, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
            ref[..., c] = bt[i, j].real
        for c in range(3):
            ref[..., 6 + 2 * c] = (b[c] * rot).real / ref_rms
            ref[..., 7 + 2 * c] = (b[c] * rot).imag / ref_rms
        ref[..., 12], ref[..., 13] = k0h.real, k0h.imag
        got = host(xd.float()).astype(np.float64)
        # both sides round the same value to bfloat16: equal up to one bf16 step at a tie
        assert np.all(np.abs(got - cnn.bf16(ref)) <= 2.0 ** -8 * np.abs(ref) + 1e-30)
        assert np.mean(got == cnn.bf16(ref)) > 0.999
        ty = np.zeros((nz, ny, nx, 6))
        for c in range(3):
            ty[..., 2 * c] = ((E[c] - b[c]) * rot).real / ref_rms
            ty[..., 2 * c + 1] = ((E[c] - b[c]) * rot).imag / ref_rms
        assert rel(host(yd).astype(np.float64), ty) < 1e-6
        xd2 = torch.empty_like(xd)
        ie.ie_nn_features(ctx, dev(p.sigma6), dev(b * np.exp(0.7j)), xd2)
        d = host((xd2.float() - xd.float()).abs()).max()
        # invariant up to the sign of the half-angle phase and rounding
        flip = host((xd2.float()[..., 6:12] + xd.float()[..., 6:12]).abs()).max()
        assert d <= 2.0 ** -7 * np.abs(ref).max() or flip <= 2.0 ** -7 * np.abs(ref).max()
    finally:
        ie.ie_ctx_destroy(ctx)


@pytest.mark.parametrize("default", ["exact", "garbage", "background"])
def test_guess_judge_takes_smallest_residual(torch, default):
    """With all weights zero the network output is zero, so the learned guess is b itself; the
    judge must keep whichever of {b, default, 0} has the smallest residual."""
    import synth
    from oracle import dense, green, operator
    from paper_2306_17537_amd import ie
    from tests.gpu_common import context, field_shape
    p = synth.random_problem((8, 8, 8), seed=5, freq=2.0e6, contrast=5.0)
    banner(f"nn judge default={default}")
    ctx, _ = context(p)
    nn = ie.ie_nn_create(14, 6, 4, 2, 0)
    try:
        ie.ie_nn_set_params(nn, np.zeros(ie.ie_nn_num_params(nn), dtype=np.float32))
        k0 = green.wavenumber(p.sigma0, p.freq)
        dsig = operator.contrast(p.sigma6, p.sigma0)
        b = _rand_field(field_shape(p), 3)
        Ghat = green.kernel_spectrum(p.n, p.h, k0, p.sigma0)
        x_ex = dense.dense_solve(p.n, p.h, p.origin, k0, p.sigma0, dsig, b)
        x0 = {"exact": x_ex, "garbage": 50.0 * _rand_field(field_shape(p), 4),
              "background": b * 0.5}[default]
        xl = b  # zero network output: the learned guess is b itself
        res = {k: np.linalg.norm(b - operator.apply_A(Ghat, dsig, v, p.n))
               for k, v in (("learned", xl), ("default", x0), ("zero", 0 * b))}
        want = {"learned": 1, "default": 0, "zero": 2}[min(res, key=res.get)]
        xd = dev(x0)
        acc = ie.ie_nn_guess(ctx, nn, dev(p.sigma6), dev(b), xd)
        assert acc == want, (acc, res)
        expect = {1: xl, 0: x0, 2: 0 * b}[acc]
        assert np.allclose(host(xd), expect, rtol=0, atol=1e-12 * np.max(np.abs(b)))
    finally:
        ie.ie_nn_destroy(nn)
        ie.ie_ctx_destroy(ctx)


@pytest.mark.parametrize("scheme", ["gs", "jacobi"])
def test_dd_with_learned_first_sweep_reaches_the_same_field(torch, scheme):
    """An untrained network may be accepted or rejected block by block; either way the DD
    solve must converge to the background-start result."""
    import synth
    from paper_2306_17537_amd import ie
    from tests.gpu_common import context, field_shape
    p = synth.random_problem((8, 8, 8), seed=6, freq=2.0e6, contrast=3.0, z_bounds=(0, 4, 8))
    banner(f"dd learned first sweep scheme={scheme}")
    ctx, g = context(p, z_bounds=(0, 4, 8))
    nn = ie.ie_nn_create(14, 6, 4, 2, 9)
    try:
        out = {}
        for init in (ie.IE_INIT_BACKGROUND, ie.IE_INIT_LEARNED):
            E = torch.zeros(field_shape(p), dtype=torch.complex128, device="cuda:0")
            opts = ie.dd_opts(scheme=ie.IE_GS if scheme == "gs" else ie.IE_JACOBI, tol=1e-8,
                              adaptive=False, inner_tol_fixed=1e-9, init=init,
                              nn=nn if init == ie.IE_INIT_LEARNED else None)
            _, st = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=dev(p.sigma6), sources=p.sources,
                                                E_total=E)], opts)
            assert st[0].relres[st[0].sweeps] <= 1e-8
            out[init] = host(E)
            banner(f"  init={init} sweeps={st[0].sweeps} its={st[0].total_its} "
                   f"learned_used={st[0].learned_used}")
        assert rel(out[ie.IE_INIT_LEARNED], out[ie.IE_INIT_BACKGROUND]) < 1e-6
    finally:
        ie.ie_nn_destroy(nn)
        ie.ie_ctx_destroy(ctx)


def test_dd_learned_rejects_bad_shapes_and_missing_network(torch):
    import synth
    from paper_2306_17537_amd import ie
    from tests.gpu_common import context, field_shape
    p = synth.random_problem((8, 8, 6), seed=6, z_bounds=(0, 3, 6))
    ctx, g = context(p, z_bounds=(0, 3, 6))
    nn = ie.ie_nn_create(14, 6, 4, 2, 9)
    try:
        E = torch.zeros(field_shape(p), dtype=torch.complex128, device="cuda:0")
        prob = [dict(grid=g, sigma6=dev(p.sigma6), sources=p.sources, E_total=E)]
        with pytest.raises(ie.IEError, match="divisible"):
            ie.ie_dd_solve([ctx], prob, ie.dd_opts(init=ie.IE_INIT_LEARNED, nn=nn))
        with pytest.raises(ie.IEError, match="ie_nn handle"):
            ie.ie_dd_solve([ctx], prob, ie.dd_opts(init=ie.IE_INIT_LEARNED))
    finally:
        ie.ie_nn_destroy(nn)
        ie.ie_ctx_destroy(ctx)
