"""The allocation-free operator call, ie_matvec_noalloc, through the C ABI: on two calls in a row
(the second on a smaller grid, both with ragged tails) it returns exactly what ie_matvec returns
for every form in both precisions, the calls leave the device's free memory unchanged, and a
grid whose scratch would not fit the fixed array is rejected."""
import numpy as np
import pytest

import synth
from tests.gpu_common import banner, context, dev, field_shape

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def test_noalloc_matvec_equals_matvec_on_two_calls_in_a_row(torch):
    from paper_2306_17537_amd import ie
    shapes = [(40, 36, 44), (9, 7, 5)]
    probs = [synth.random_problem(n, seed=11 + k, freq=2.0e6, contrast=3.0)
             for k, n in enumerate(shapes)]
    ctxs = [context(p)[0] for p in probs]
    try:
        s6 = [dev(p.sigma6) for p in probs]
        forms = (ie.IE_CONVENTIONAL, ie.IE_CIE, ie.IE_GREEN_ONLY, ie.IE_SCATTER)
        for prec, dt in ((ie.IE_FP64, torch.complex128), (ie.IE_MIXED, torch.complex64)):
            for form in forms:
                xs = [dev(_rand(field_shape(p), 3 + k)).to(dt) for k, p in enumerate(probs)]
                refs = []
                for k in range(2):
                    y = torch.zeros_like(xs[k])
                    ie.ie_matvec(ctxs[k], s6[k], xs[k], y, form, prec)
                    refs.append(y)
                torch.cuda.synchronize()
                ie.ie_matvec_noalloc(ctxs[1], s6[1], xs[1], torch.empty_like(xs[1]), form, prec)
                torch.cuda.synchronize()
                free0 = torch.cuda.mem_get_info()[0]
                outs = []
                for k in range(2):  # the larger grid, then the smaller one
                    banner(f"noalloc prec={prec} form={form} n={probs[k].n}")
                    y = torch.full_like(xs[k], complex(float("nan"), float("nan")))
                    ie.ie_matvec_noalloc(ctxs[k], s6[k], xs[k], y, form, prec)
                    torch.cuda.synchronize()
                    outs.append(y)
                free1 = torch.cuda.mem_get_info()[0]
                assert free1 == free0, (prec, form, free0 - free1)
                for k in range(2):
                    assert torch.equal(outs[k], refs[k]), (prec, form, probs[k].n)
    finally:
        for c in ctxs:
            ie.ie_ctx_destroy(c)


def test_noalloc_rejects_a_grid_beyond_the_fixed_array(torch):
    from paper_2306_17537_amd import ie
    p = synth.random_problem((64, 64, 64), seed=5, freq=2.0e6, contrast=1.0)
    ctx, _ = context(p, mask=ie.IE_FP64 | ie.IE_MIXED)
    try:
        s6 = dev(p.sigma6)
        x = dev(_rand(field_shape(p), 1))
        y = torch.zeros_like(x)
        with pytest.raises(ie.IEError) as err:
            ie.ie_matvec_noalloc(ctx, s6, x, y, ie.IE_CONVENTIONAL, ie.IE_FP64)
        assert err.value.code == ie.IE_EINVAL and "scratch" in str(err.value)
        # the same grid in complex64 fits and equals ie_matvec
        x32 = x.to(torch.complex64)
        y_ref = torch.zeros_like(x32)
        ie.ie_matvec(ctx, s6, x32, y_ref, ie.IE_CIE, ie.IE_MIXED)
        y32 = torch.zeros_like(x32)
        ie.ie_matvec_noalloc(ctx, s6, x32, y32, ie.IE_CIE, ie.IE_MIXED)
        torch.cuda.synchronize()
        assert torch.equal(y32, y_ref)
    finally:
        ie.ie_ctx_destroy(ctx)
