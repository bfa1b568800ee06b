"""Acceptance test from the isolated sub-domains example (sec. 3.1): two 0.01 S/m anomalies in a
0.1 S/m background on a 128^3 grid, 24 kHz, conventional form, GMRES(10) to e = 1e-6.  Block
Gauss-Seidel over the partition [background | anomaly | background | anomaly | background]
(zero-contrast blocks take no inner iterations, E_i = b_i) must give the full-domain result:
the paper reports the magnetic fields of both within 0.01 % average normalised magnitude
difference.  Both are checked against the oracle's solve of the same problem."""
import os

import numpy as np
import pytest

import synth
from tests.gpu_common import banner, context, dev, field_shape, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_dd_equals_full_domain_on_two_isolated_anomalies(torch):
    from paper_2306_17537_amd import ie
    p = synth.example1()
    banner(f"example 1: {p.n}, partition {p.z_bounds}")
    ctx, g = context(p, z_bounds=p.z_bounds)
    try:
        s6 = dev(p.sigma6)
        shape = field_shape(p)
        E0 = torch.empty(shape, dtype=torch.complex128, device="cuda:0")
        ie.ie_background_field(ctx, p.sources, E0)
        Ef = E0.clone()
        _, gst = ie.ie_gmres(ctx, s6, E0, Ef, tol=1e-6, restart=10, precision=ie.IE_FP64,
                             form=ie.IE_CONVENTIONAL)
        Et = Ef.clone()  # the same solve continued to e = 1e-10
        ie.ie_gmres(ctx, s6, E0, Et, tol=1e-10, restart=10, precision=ie.IE_FP64,
                    form=ie.IE_CONVENTIONAL)
        Ed = torch.zeros(shape, dtype=torch.complex128, device="cuda:0")
        opts = ie.dd_opts(scheme=ie.IE_GS, adaptive=False, tol=1e-6, inner_tol_fixed=1e-6,
                          precision=ie.IE_FP64, form=ie.IE_CONVENTIONAL, max_sweeps=30)
        _, st = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=s6, sources=p.sources, E_total=Ed)],
                               opts)
        st = st[0]
        its_blocks = [[st.block_its[k][i] for i in range(st.nblocks)] for k in range(st.sweeps)]
        banner(f"  full domain: {gst.its} GMRES iterations, relres {gst.relres:.2e}")
        banner(f"  block GS: {st.sweeps} sweeps, {st.total_its} inner iterations "
               f"{its_blocks}, relres {st.relres[st.sweeps]:.2e}")
        assert gst.relres <= 1e-6 and st.relres[st.sweeps] <= 1e-6
        # zero-contrast blocks never iterate
        assert all(row[0] == 0 and row[2] == 0 and row[4] == 0 for row in its_blocks)
        # the oracle's solve to e <= 1e-10 (make_golden.py): E - E0 at sampled cells of the
        # anomalies and H at 20 receivers on lines through and between them
        d = np.load(os.path.join(os.path.dirname(__file__), "golden", "example1_sample.npz"))
        e0 = host(E0).reshape(3, -1)[:, d["idx"]]

        def err(E):
            Ea = host(E).reshape(3, -1)[:, d["idx"]] - e0
            return float(np.linalg.norm(Ea - d["Ea"]) / np.linalg.norm(d["Ea"]))

        def h_err(E):
            H, _ = ie.ie_receivers(ctx, s6, p.sources, E, d["rx"])
            return float(np.mean(np.linalg.norm(H - d["H_total"], axis=1) /
                                 np.linalg.norm(d["H_total"], axis=1))), H

        et, ef, ed = err(Et), err(Ef), err(Ed)
        (ht, _), (hf, Hf), (hd, Hd) = h_err(Et), h_err(Ef), h_err(Ed)
        diff = np.mean(np.linalg.norm(Hd - Hf, axis=1) / np.linalg.norm(Hf, axis=1))
        banner(f"  E - E0 in the anomalies vs the oracle: e=1e-10 solve {et:.2e}, block GS "
               f"{ed:.2e}, full domain {ef:.2e}; H vs the oracle (mean normalised): {ht:.2e}, "
               f"{hd:.2e}, {hf:.2e}; block GS vs full domain {diff:.2e}")
        assert et < 1e-6
        assert diff < 1e-4 and hd < 1e-4 and hf < 1e-4  # the paper's criterion: 0.01 %
        # both iterates stop at e = 1e-6; inside the resistive bodies that leaves errors of
        # order 1e-3 (measured), the same for either method
        assert ed < 2e-3 and ef < 2e-3
    finally:
        ie.ie_ctx_destroy(ctx)
