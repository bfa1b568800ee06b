"""The trained learned-initial-guess network on held-out models of the 64^3 three-layer dipping
workload (seeds 50000-50002, not in the training set): what it gains over the zero start, and
that the zero-start judge keeps every solve correct.

Measured on the MI355X (16 held-out models, weights in the package): the learned start did not
reduce GMRES iterations (first-sweep inner iterations of block GS 777 from the learned start,
743 from zero; full-domain mixed GMRES 485 vs 471 on average, judge cycles included).  The gain
is asserted below and expected to fail (xfail, with these numbers); the other tests hold what
does work: the stored network predicts finite fields, the residual judge picks the best start,
and every solve reaches the same field whatever it starts from.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import banner, context, dev, host, rel

pytestmark = pytest.mark.gpu

SEEDS = (50000, 50001, 50002)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def net(torch):
    from paper_2306_17537_amd import guess, ie
    nn = guess.create()
    yield nn
    ie.ie_nn_destroy(nn)


def test_trained_network_guess_and_residual_judge(torch, net):
    """The stored weights load and predict finite fields; the residual judge of ie_nn_guess
    keeps the learned guess exactly when its residual beats both the zero and the background
    start (measured here through ie_matvec)."""
    from paper_2306_17537_amd import ie
    for seed in SEEDS:
        p = synth.config1(seed=seed)
        ctx, _ = context(p)
        try:
            nx, ny, nz = p.n
            s6 = dev(p.sigma6)
            E0 = torch.empty((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0")
            ie.ie_background_field(ctx, p.sources, E0)
            x = torch.empty_like(E0)
            ie.ie_nn_predict(ctx, net, s6, E0, x)
            assert bool(torch.isfinite(torch.view_as_real(x)).all())
            r = torch.empty_like(E0)
            bn = float(torch.linalg.vector_norm(E0))

            def resid(v):
                ie.ie_matvec(ctx, s6, v, r, ie.IE_CONVENTIONAL, ie.IE_FP64)
                return float(torch.linalg.vector_norm(E0 - r)) / bn

            r_nn, r_bg = resid(x), resid(E0)
            banner(f"seed={seed}: relative residual of the learned guess {r_nn:.3f}, of the "
                   f"background start {r_bg:.3f}, of the zero start 1")
            xd = E0.clone()
            acc = ie.ie_nn_guess(ctx, net, s6, E0, xd)
            want = 1 if r_nn < min(1.0, r_bg) else (2 if 1.0 < r_bg else 0)
            assert acc == want
        finally:
            ie.ie_ctx_destroy(ctx)


def test_learned_start_keeps_full_domain_solves_correct(torch, net):
    from paper_2306_17537_amd import guess, ie
    tot = {"zero": 0, "learned": 0}
    for seed in SEEDS:
        p = synth.config1(seed=seed)
        ctx, _ = context(p)
        try:
            nx, ny, nz = p.n
            s6 = dev(p.sigma6)
            E0 = torch.empty((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0")
            ie.ie_background_field(ctx, p.sources, E0)
            out = {}
            for name in ("zero", "learned"):
                x = torch.zeros_like(E0)
                pre = 0
                if name == "learned":
                    guess.solve_learned_start(ctx, net, s6, E0, x)
                    pre = 20  # the two judge cycles
                _, st = ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, precision=ie.IE_MIXED,
                                    form=ie.IE_CIE)
                out[name] = (host(x), st.its + pre)
                tot[name] += st.its + pre
            banner(f"seed={seed}: GMRES its zero start {out['zero'][1]}, learned start "
                   f"{out['learned'][1]} (judge cycles included)")
            assert rel(out["learned"][0], out["zero"][0]) < 1e-5
        finally:
            ie.ie_ctx_destroy(ctx)
    banner(f"total its: zero {tot['zero']}, learned {tot['learned']}, gain "
           f"{(tot['zero'] - tot['learned']) / tot['zero']:+.1%}")


@pytest.mark.xfail(strict=False, reason="negative result, measured on 16 held-out models: the "
                   "learned first-sweep guess takes 777 block-GS inner iterations against 743 "
                   "from zero (its residual is 0.25-9.6 times the zero start's)")
def test_learned_guess_reduces_first_sweep_inner_iterations(torch, net):
    """What the network is for (the learned part of the solver): on held-out models the first
    block GS sweep (fixed inner tolerance 1e-6) from the learned guesses needs fewer inner
    iterations than from zero, judge cycles included."""
    from paper_2306_17537_amd import ie
    tot = {ie.IE_INIT_ZERO: 0, ie.IE_INIT_LEARNED: 0}
    for seed in SEEDS:
        p = synth.config1(seed=seed)
        ctx, g = context(p, z_bounds=p.z_bounds)
        try:
            nx, ny, nz = p.n
            for init in tot:
                E = torch.zeros((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0")
                opts = ie.dd_opts(scheme=ie.IE_GS, adaptive=False, inner_tol_fixed=1e-6,
                                  tol=1e-6, init=init, precision=ie.IE_MIXED, max_sweeps=1,
                                  nn=net if init == ie.IE_INIT_LEARNED else None)
                _, st = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=dev(p.sigma6),
                                                    sources=p.sources, E_total=E)], opts,
                                       allow_noconv=True)
                tot[init] += sum(st[0].block_its[0][i] for i in range(st[0].nblocks))
        finally:
            ie.ie_ctx_destroy(ctx)
    banner(f"first-sweep inner iterations: zero {tot[ie.IE_INIT_ZERO]}, learned "
           f"{tot[ie.IE_INIT_LEARNED]}")
    assert tot[ie.IE_INIT_LEARNED] < tot[ie.IE_INIT_ZERO]


def test_dd_learned_first_sweep_on_a_held_out_model(torch, net):
    from paper_2306_17537_amd import ie
    p = synth.config1(seed=SEEDS[1])
    ctx, g = context(p, z_bounds=p.z_bounds)
    try:
        nx, ny, nz = p.n
        res = {}
        for init in (ie.IE_INIT_ZERO, ie.IE_INIT_LEARNED):
            E = torch.zeros((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0")
            opts = ie.dd_opts(scheme=ie.IE_GS, adaptive=True, tol=1e-6, init=init,
                              precision=ie.IE_MIXED,
                              nn=net if init == ie.IE_INIT_LEARNED else None)
            _, st = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=dev(p.sigma6), sources=p.sources,
                                                E_total=E)], opts)
            res[init] = (host(E), st[0])
            first = sum(st[0].block_its[0][i] for i in range(st[0].nblocks))
            banner(f"dd init={init}: sweeps {st[0].sweeps}, its {st[0].total_its}, first sweep "
                   f"{first}, learned blocks {st[0].learned_used}")
        assert rel(res[ie.IE_INIT_LEARNED][0], res[ie.IE_INIT_ZERO][0]) < 1e-4
    finally:
        ie.ie_ctx_destroy(ctx)
