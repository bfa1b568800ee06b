"""Write stored reference fields for the GPU parity tests and the bench accuracy check.

Calls only the CPU oracle (oracle/) on the seeded synthetic inputs of synth/.  Every file holds
the oracle's full-domain solve (contraction form, restarted GMRES) to relative residual
<= 1e-10 (eq. 9):

* ``config1_Ea.npz``: the whole anomalous field E - E0 of the 64^3 workload as complex64 (the
  stored precision, ~1e-7 relative, is far below the 1e-4 parity gate), the oracle's relative
  residual and the norm of E0;
* ``<name>_sample.npz`` for grids too large to store whole: E - E0 (complex128) at a seeded
  sample of cells plus every cell of the central z column, the magnetic field (total and
  scattered, eqs. 4 and 6) at receiver points, and the norms of E0 and of the whole E - E0.

    python tests/golden/make_golden.py config1 example1 config2 config3
"""
import os
import sys
import time

import numpy as np
import scipy.fft

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import receivers, solve  # noqa: E402

WORKERS = os.cpu_count() or 1


def _solve(problem, tol, restart):
    st = solve.setup(problem)
    with scipy.fft.set_workers(WORKERS):
        E, info = solve.solve_full(st, form="cie", tol=tol, restart=restart, max_its=20000)
    return st, E, info


def make(name, problem, tol=1e-10):
    t0 = time.time()
    st, E, info = _solve(problem, tol, 10)
    Ea = (E - st.E0).astype(np.complex64)
    out = os.path.join(HERE, f"{name}_Ea.npz")
    np.savez_compressed(out, Ea=Ea, relres=info["relres_eq9"], e0norm=np.linalg.norm(st.E0),
                        its=info["its"], tol=tol)
    print(f"{name}: its={info['its']} relres={info['relres_eq9']:.2e} "
          f"t={time.time() - t0:.0f}s -> {out}", flush=True)


def sample_cells(n, nsample, seed, mask=None):
    """Flat [nz][ny][nx] indices: ``nsample`` distinct cells drawn with PCG64(seed) (from the
    cells where ``mask`` is true, if given) plus the central z column, sorted."""
    nx, ny, nz = n
    pool = np.arange(nx * ny * nz) if mask is None else np.flatnonzero(mask.ravel())
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.choice(pool, size=min(nsample, pool.size), replace=False)
    column = np.arange(nz) * (nx * ny) + (ny // 2) * nx + nx // 2
    if mask is not None:
        column = column[mask.ravel()[column]]
    return np.unique(np.concatenate([pick, column])).astype(np.int64)


def make_sampled(name, problem, rx=(), tol=1e-10, restart=10, nsample=4096, seed=7,
                 anomalous_only=False):
    t0 = time.time()
    st, E, info = _solve(problem, tol, restart)
    t_solve = time.time() - t0
    Ea = E - st.E0
    mask = np.any(st.dsig.reshape(9, -1) != 0, axis=0).reshape(st.E0.shape[1:]) \
        if anomalous_only else None
    idx = sample_cells(problem.n, nsample, seed, mask)
    rx = np.asarray(rx, dtype=np.float64).reshape(-1, 3)
    if len(rx):
        Ht = receivers.h_total(problem.n, problem.h, problem.origin, st.dsig, E, rx,
                               problem.sources, st.k0, st.sigma0)
        Ha = receivers.h_anomalous(problem.n, problem.h, problem.origin, st.dsig, E, rx, st.k0)
    else:
        Ht = Ha = np.zeros((0, 3), dtype=np.complex128)
    out = os.path.join(HERE, f"{name}_sample.npz")
    np.savez_compressed(out, idx=idx, Ea=Ea.reshape(3, -1)[:, idx], rx=rx, H_total=Ht,
                        H_anom=Ha, relres=info["relres_eq9"], its=info["its"], tol=tol,
                        restart=restart, e0norm=np.linalg.norm(st.E0),
                        ea_norm=np.linalg.norm(Ea), n=np.array(problem.n),
                        solve_s=t_solve, problem=problem.name)
    print(f"{name}: its={info['its']} relres={info['relres_eq9']:.2e} "
          f"solve {t_solve:.0f}s, total {time.time() - t0:.0f}s -> {out}", flush=True)


# magnetic-field receivers 7, 15 and 30 m from the transmitter along the tool (z) axis
LOG_RX = [[0.0, 0.0, 7.0], [0.0, 0.0, 15.0], [0.0, 0.0, 30.0]]
# a line of receivers through and between the two anomalies of the isolated sub-domains example
EX1_RX = [[x, 0.0, z] for z in (-15.0, -8.0, 0.5, 8.0, 15.0) for x in (-10.0, -3.0, 2.0, 9.0)]


def config2_group_members():
    """Index (in synth.config2() order) of the first problem of each (grid shape, frequency)."""
    seen = {}
    for k, p in enumerate(synth.config2()):
        seen.setdefault((p.n, p.freq), k)
    return sorted(seen.values())


if __name__ == "__main__":
    which = sys.argv[1:] or ["config1"]
    for w in which:
        if w == "config1":
            make("config1", synth.config1())
        elif w == "example1":
            make_sampled("example1", synth.example1(), rx=EX1_RX, anomalous_only=True)
        elif w == "config2":
            probs = synth.config2()
            for k in config2_group_members():
                p = probs[k]
                make_sampled(f"config2_member{k:03d}", p, rx=LOG_RX[:1], nsample=2048)
        elif w == "config3":
            make_sampled("config3", synth.config3(), rx=LOG_RX, restart=30)
        else:
            raise SystemExit(f"unknown workload {w}")
