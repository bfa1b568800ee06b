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
