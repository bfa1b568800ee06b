"""The stored oracle reference fields (tests/golden/*.npz, written by make_golden.py from the
oracle only) satisfy the oracle's own residual check."""
import os

import numpy as np
import pytest
import scipy.fft

import synth
from oracle import operator, solve

HERE = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.slow
def test_config1_reference_satisfies_eq9():
    d = np.load(os.path.join(HERE, "config1_Ea.npz"))
    assert float(d["relres"]) <= 1e-10
    p = synth.config1()
    st = solve.setup(p)
    E = st.E0 + d["Ea"].astype(np.complex128)
    with scipy.fft.set_workers(os.cpu_count() or 1):
        e = operator.relres(st.Ghat, st.dsig, E, st.E0, p.n)
    # complex64 storage of the field limits the recomputed residual to ~1e-7
    assert e < 1e-6
    assert np.isclose(np.linalg.norm(st.E0), float(d["e0norm"]), rtol=1e-12)


def _sampled_references():
    names = sorted(f[:-len("_sample.npz")] for f in os.listdir(HERE) if f.endswith("_sample.npz"))
    return names


def _problem(name):
    if name == "config3":
        return synth.config3()
    if name == "example1":
        return synth.example1()
    if name.startswith("config2_member"):
        return synth.config2()[int(name[len("config2_member"):])]
    raise KeyError(name)


@pytest.mark.parametrize("name", _sampled_references())
def test_sampled_reference_is_consistent_with_its_problem(name):
    """Each sampled reference records a converged oracle solve (relative residual <= 1e-10 by
    eq. 9) of the problem it names: the background-field norm matches the oracle's E0 of that
    problem, the sample indexes distinct cells of its grid, and H_total - H_anom at the
    receivers is the oracle's background field there (eqs. 4, 6)."""
    from oracle import green, receivers, source
    d = np.load(os.path.join(HERE, f"{name}_sample.npz"))
    p = _problem(name)
    assert str(d["problem"]) == p.name
    assert tuple(int(v) for v in d["n"]) == tuple(p.n)
    assert float(d["relres"]) <= 1.0001e-10 and int(d["its"]) > 0
    nx, ny, nz = p.n
    idx = d["idx"]
    assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < nx * ny * nz
    assert d["Ea"].shape == (3, idx.size) and np.all(np.isfinite(d["Ea"]))
    assert 0 < np.linalg.norm(d["Ea"]) <= float(d["ea_norm"])
    k0 = green.wavenumber(p.sigma0, p.freq)
    E0 = source.background_field(p.n, p.h, p.origin, p.sources, k0, p.freq, p.sigma0)
    assert np.isclose(np.linalg.norm(E0), float(d["e0norm"]), rtol=1e-12)
    if d["rx"].size:
        H0 = receivers.h_background(d["rx"], p.sources, k0, p.sigma0)
        assert np.allclose(d["H_total"] - d["H_anom"], H0, rtol=1e-12, atol=0)
