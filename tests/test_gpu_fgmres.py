"""GPU parity of the Krylov outer iteration over the DD sweep (flexible GMRES, right-
preconditioned by one block Gauss-Seidel or Jacobi sweep) against the CPU oracle: the dense
solution and the oracle's outer step counts on small grids, and the stored oracle field on the
64^3 workload."""
import os

import numpy as np
import pytest

import synth
from oracle import dd, dense, solve
from tests.gpu_common import banner, context, dev, field_shape, host, rel

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("scheme", ["gs", "jacobi"])
@pytest.mark.parametrize("zb", [(0, 4, 8), (0, 2, 5, 8)])
def test_fgmres_dd_small_matches_oracle(torch, scheme, zb):
    from paper_2306_17537_amd import ie
    p = synth.random_problem((8, 8, 8), seed=9, freq=2.0e6, contrast=3.0, z_bounds=zb)
    banner(f"fgmres-dd {scheme} partition {zb}")
    st = solve.setup(p)
    ref = dense.dense_solve(p.n, p.h, p.origin, st.k0, p.sigma0, st.dsig, st.E0)
    _, oinfo = dd.fgmres_dd(st, zb, scheme, tol=1e-10, inner_tol=1e-3, form="cie")
    ctx, g = context(p, z_bounds=zb)
    try:
        E = torch.zeros(field_shape(p), dtype=torch.complex128, device="cuda:0")
        opts = ie.dd_opts(scheme=ie.IE_FGMRES_GS if scheme == "gs" else ie.IE_FGMRES_JACOBI,
                          tol=1e-10, inner_tol_fixed=1e-3, init=ie.IE_INIT_ZERO,
                          precision=ie.IE_FP64, form=ie.IE_CIE, max_sweeps=100)
        _, s = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=dev(p.sigma6), sources=p.sources,
                                           E_total=E)], opts)
        s = s[0]
        banner(f"  GPU outer {s.sweeps} inner {s.total_its} relres {s.relres[s.sweeps]:.2e}; "
               f"oracle outer {oinfo['its']} inner {oinfo['inner_its']}")
        assert s.relres[s.sweeps] <= 1e-10
        assert rel(host(E), ref) < 1e-8
        assert abs(s.sweeps - oinfo["its"]) <= 2
    finally:
        ie.ie_ctx_destroy(ctx)


@pytest.mark.parametrize("scheme", ["gs", "jacobi"])
def test_fgmres_dd_full_size_matches_stored_oracle_field(torch, scheme):
    from paper_2306_17537_amd import ie
    p = synth.config1()
    banner(f"fgmres-dd full size {scheme}")
    gold = np.load(os.path.join(ROOT, "tests", "golden", "config1_Ea.npz"))["Ea"].astype(np.complex128)
    ctx, g = context(p, z_bounds=p.z_bounds)
    try:
        E = torch.zeros(field_shape(p), dtype=torch.complex128, device="cuda:0")
        Ea = torch.zeros_like(E)
        opts = ie.dd_opts(scheme=ie.IE_FGMRES_GS if scheme == "gs" else ie.IE_FGMRES_JACOBI,
                          tol=1e-6, inner_tol_fixed=1e-2, init=ie.IE_INIT_ZERO,
                          precision=ie.IE_MIXED, form=ie.IE_CIE, max_sweeps=120)
        _, s = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=dev(p.sigma6), sources=p.sources,
                                           E_total=E, E_anom=Ea)], opts)
        s = s[0]
        err = rel(host(Ea), gold)
        banner(f"  outer {s.sweeps}, inner {s.total_its}, relres {s.relres[s.sweeps]:.2e}, "
               f"{s.seconds * 1e3:.1f} ms, Ea rel err {err:.2e}")
        assert s.relres[s.sweeps] <= 1e-6
        assert err < 1e-4
    finally:
        ie.ie_ctx_destroy(ctx)


def test_fgmres_rejects_learned_start_and_zero_inner_tolerance(torch):
    from paper_2306_17537_amd import ie
    p = synth.random_problem((4, 4, 4), seed=1, z_bounds=(0, 2, 4))
    ctx, g = context(p, z_bounds=(0, 2, 4))
    try:
        E = torch.zeros(field_shape(p), dtype=torch.complex128, device="cuda:0")
        prob = [dict(grid=g, sigma6=dev(p.sigma6), sources=p.sources, E_total=E)]
        with pytest.raises(ie.IEError, match="inner_tol_fixed"):
            ie.ie_dd_solve([ctx], prob, ie.dd_opts(scheme=ie.IE_FGMRES_GS, inner_tol_fixed=0.0))
        with pytest.raises(ie.IEError, match="learned"):
            ie.ie_dd_solve([ctx], prob, ie.dd_opts(scheme=ie.IE_FGMRES_GS,
                                                   init=ie.IE_INIT_LEARNED))
    finally:
        ie.ie_ctx_destroy(ctx)
