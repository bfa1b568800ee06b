"""Write stored reference fields for the GPU parity tests and the bench accuracy check.

Calls only the CPU oracle (oracle/) on the seeded synthetic inputs of synth/.  Each file holds
the anomalous field E - E0 of the oracle's full-domain solve (contraction form, restarted GMRES
with restart 10) to relative residual <= 1e-10 (eq. 9), stored as complex64 (the stored
precision, ~1e-7 relative, is far below the 1e-4 parity gate), plus the oracle's own relative
residual and the norm of E0.

    python tests/golden/make_golden.py config1
"""
import os
import sys
import time

import numpy as np
import scipy.fft

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import solve  # noqa: E402


def make(name, problem, tol=1e-10):
    t0 = time.time()
    st = solve.setup(problem)
    with scipy.fft.set_workers(os.cpu_count() or 1):
        E, info = solve.solve_full(st, form="cie", tol=tol, max_its=20000)
    Ea = (E - st.E0).astype(np.complex64)
    out = os.path.join(HERE, f"{name}_Ea.npz")
    np.savez_compressed(out, Ea=Ea, relres=info["relres_eq9"], e0norm=np.linalg.norm(st.E0),
                        its=info["its"], tol=tol)
    print(f"{name}: its={info['its']} relres={info['relres_eq9']:.2e} "
          f"t={time.time() - t0:.0f}s -> {out}", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["config1"]
    for w in which:
        if w == "config1":
            make("config1", synth.config1())
        else:
            raise SystemExit(f"unknown workload {w}")
