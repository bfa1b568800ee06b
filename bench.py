#!/usr/bin/env python3
"""Benchmark of the integral-equation solver on one MI355X.

Workload (one "step"): one complete solve of the 128x128x256 six-layer dipping TI model (cell
0.25 m, 12.6 M complex unknowns, principal conductivities in [0.1, 10] S/m, 2 MHz, z dipole at
the centre) to full-domain relative residual 1e-6 (eq. 9) by the plain float64 method:
background field, contrast preparation and restarted GMRES on the contraction form in complex128
from a zero start.  The Green's spectrum is built once before the timed region (it depends on
grid and medium only) and timed separately.  Beside it, on the same grid: the chosen form
(complex64 Krylov vectors and convolutions, float64 residual at every restart, Arnoldi scalars,
Givens rotations and solution accumulation), the Krylov outer iteration over block sweeps and
stationary block Gauss-Seidel over four z slabs, each with its anomalous-field error against the
stored oracle reference.

Printed: one JSON line with the contract fields plus
  roofline     - dominant kernel of the timed solve: algorithmic bytes / duration from HIP events
                 on the launch stream (library launch profiler, a replay of the step), against
                 8 TB/s, with the rocprofv3 average of the same kernel from the committed
                 kernel-trace summary when it was measured on the current kernel sources;
  roofline_alu - the same kernel against the non-packed vector-ALU peak (model flops: 5 L log2 L
                 per transform, 72 per point for the tensor multiply);
  cpu_baseline - the CPU oracle on this host, sampled and scaled to one solve;
  chosen_form  - the mixed-precision solve on the same grid, its speed-up and field error;
  solve_large  - the block forms on the same grid;
  config1      - the 64^3 three-layer model: chosen form, plain float64, block GS / Jacobi;
  accuracy     - relative L2 errors of the anomalous field against the stored oracle references.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solve @ rel.resid 1e-6 + matvec HBM GB/s; plain FP64 vs mixed+NN"
HBM_PEAK_GBS = 8000.0
# Non-packed vector peak (packed FP32 instructions are disabled in the build): 256 CUs x 4 SIMDs x
# 16 lanes x 2 flop (FMA) x 2.4 GHz, the same for float32 and float64.
VALU_PEAK_TFLOPS = 78.6
# Restart length of the timed forms.  The paper runs GMRES(10).  In mixed precision, summed over
# the 64^3 model and four held-out seeds of it, restart 16 took 6 % less time than 10 and 2 % less
# than 12 (fewer restarts, each a float64 residual; fewer Arnoldi steps).  Plain float64 is also
# timed at 10.
CHOSEN_RESTART = 16    # the chosen (mixed) form
HEADLINE_RESTART = 10  # the plain float64 method: the paper's restart length (sec. 3.1)
LARGE_WORKLOAD = ("128x128x256 cells of 0.25 m (12.6 M complex unknowns), six tilted-TI layers "
                  "dipping 20 deg, principal conductivities 0.1-10 S/m (seed 303), 2 MHz, z "
                  "dipole at the centre")


# launch variants measured by the autotuner on this GPU for every grid the benchmark sets up
# (written by a run with --tuning none --save-tuning), so that repeated runs and the profiler
# runs time the same kernels
DEFAULT_TUNING = os.path.join(ROOT, "paper_2306_17537_amd", "tuning_gfx950.json")
# kernel-trace summary of the timed solves alone (the dominant kernel also serves other grids in
# a default run)
HEADLINE_TRACE = "large_grid_fp64_and_mixed_solves_trace.md"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the comparison forms on the 64^3 model")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-seq", type=int, default=16,
                    help="problems of the logging run also solved one call each (speed-up)")
    ap.add_argument("--profile-json", default=None, help="write the kernel profile here")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="first run the 1 GiB fill and copy kernels that scale the HBM counters")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the operator alone and the block forms on the 128x128x256 grid")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned-guess comparison")
    ap.add_argument("--no-ex1", action="store_true",
                    help="skip the isolated sub-domains example (128^3, DD vs full domain)")
    ap.add_argument("--no-small", action="store_true", help="skip the 64^3 model legs")
    ap.add_argument("--tuning", default=DEFAULT_TUNING,
                    help="launch-variant file to load before any setup ('none': tune every grid)")
    ap.add_argument("--save-tuning", default=None,
                    help="write the launch-variant cache of this run here at the end")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sample_error(E_anom, name):
    """Relative L2 error of an anomalous field (host array [3, nz, ny, nx]) against the oracle
    reference stored at sampled cells, or None if the reference file is absent."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_sample.npz")
    if not os.path.exists(path):
        return None
    d = np.load(path)
    got = E_anom.reshape(3, -1)[:, d["idx"]]
    return float(np.linalg.norm(got - d["Ea"]) / np.linalg.norm(d["Ea"]))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the solver has no "
                                   "multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import synth
    from paper_2306_17537_amd import ie

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ie.lib()
    tuning_file = None
    if args.tuning != "none" and os.path.exists(args.tuning):
        ie.ie_tuning_load(args.tuning)
        tuning_file = os.path.relpath(args.tuning, ROOT)
    if args.pmc_calibration:
        from paper_2306_17537_amd import traffic
        traffic.calibrate()
    p = synth.config3()
    nx, ny, nz = p.n
    g = ie.make_grid(p.n, p.h, p.origin)
    med = ie.ie_medium(p.sigma0, p.freq, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = ie.ie_green_setup(g, med, p.z_bounds, ie.IE_FP64 | ie.IE_MIXED)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"green setup {setup_s * 1e3:.1f} ms")
    s6 = torch.from_numpy(p.sigma6).cuda()
    shape = (3, nz, ny, nx)
    E0 = torch.zeros(shape, dtype=torch.complex128, device="cuda:0")
    x = torch.zeros_like(E0)
    Ea = torch.zeros_like(E0)

    def solve(precision, restart=HEADLINE_RESTART):
        # background field + contrast + GMRES from a zero start, all inside the timed step
        torch.cuda.synchronize()
        t = time.perf_counter()
        ie.ie_background_field(ctx, p.sources, E0)
        x.zero_()
        _, gst = ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, precision=precision, form=ie.IE_CIE,
                             restart=restart, max_its=5000)
        torch.sub(x, E0, out=Ea)
        torch.cuda.synchronize()
        return time.perf_counter() - t, gst

    for _ in range(args.warmup):
        solve(ie.IE_FP64)
    log("timed region")
    times = []
    for _ in range(args.steps):
        dt, st = solve(ie.IE_FP64)
        times.append(dt)
    total = sum(times)
    ms_per_step = 1e3 * total / args.steps
    fp64_stats = st
    acc = {"fp64_Ea_rel_err": sample_error(Ea.cpu().numpy(), "config3")}
    log(f"float64 solve: {ms_per_step:.1f} ms/solve, its={st.its} restarts={st.restarts} "
        f"relres={st.relres:.3e} error vs oracle {acc['fp64_Ea_rel_err']}")

    # the same step replayed with direct kernel launches under the library's launch profiler
    ie.ie_profile_begin()
    nprof = max(1, min(args.steps, 2))
    t_prof = [solve(ie.IE_FP64)[0] for _ in range(nprof)]
    prof = ie.ie_profile_end()
    log(f"profiled replay: {1e3 * sum(t_prof) / nprof:.1f} ms/solve")
    kern = [k for k in prof if not k["name"].startswith("finalise")]
    dom = kern[0]
    avg_ms = dom["total_ms"] / dom["launches"]
    achieved = dom["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    tuning = ie.ie_ctx_tuning(ctx)
    dom_kernel = template_name(dom["name"], tuning, p.n)
    traffic_bytes = traffic_src = rocprof = None
    if dom_kernel:
        from paper_2306_17537_amd import traffic
        hit = traffic.lookup(dom_kernel)
        if hit is not None:
            traffic_bytes, traffic_src = hit[0], os.path.relpath(hit[2], ROOT)
        tr = traffic.trace_lookup(dom_kernel, summary=HEADLINE_TRACE)
        if tr is not None:
            rocprof = dict(avg_us=tr[0], calls=tr[1], source=os.path.relpath(tr[2], ROOT),
                           achieved=round(dom["bytes_per_launch"] / (tr[0] * 1e-6) / 1e9, 1),
                           frac=round(dom["bytes_per_launch"] / (tr[0] * 1e-6) / 1e9 /
                                      HBM_PEAK_GBS, 4))
    prof_total = sum(k["total_ms"] for k in prof)
    if args.profile_json:
        with open(args.profile_json, "w") as f:
            json.dump(dict(kernels=prof, steps=nprof), f, indent=1)

    # the chosen form on the same grid
    solve(ie.IE_MIXED, CHOSEN_RESTART)
    t_mixed = []
    for _ in range(3):
        dt, cst = solve(ie.IE_MIXED, CHOSEN_RESTART)
        t_mixed.append(dt)
    acc["chosen_Ea_rel_err"] = sample_error(Ea.cpu().numpy(), "config3")
    solve(ie.IE_FP64, CHOSEN_RESTART)
    t16, st16 = solve(ie.IE_FP64, CHOSEN_RESTART)
    chosen = dict(form=f"full-domain contraction-form GMRES({CHOSEN_RESTART}) from zero, "
                       "complex64 Krylov vectors and convolutions + float64 residual, Arnoldi "
                       "scalars, Givens rotations and solution",
                  s=round(float(np.median(t_mixed)), 4), its=cst.its,
                  refinements=cst.refinements, relres=float(f"{cst.relres:.3e}"),
                  Ea_rel_err=acc["chosen_Ea_rel_err"],
                  speedup_vs_fp64=round((total / args.steps) / float(np.median(t_mixed)), 3),
                  fp64_gmres16=dict(s=round(t16, 4), its=st16.its,
                                    relres=float(f"{st16.relres:.3e}")))
    log(f"chosen form: {chosen}")

    # the paper's observable: H at receivers 7, 15 and 30 m from the transmitter (eqs. 4, 6)
    rx = [[0.0, 0.0, 7.0], [0.0, 0.0, 15.0], [0.0, 0.0, 30.0]]
    torch.cuda.synchronize()
    t = time.perf_counter()
    H, Ha = ie.ie_receivers(ctx, s6, p.sources, x, rx)
    t_rx = time.perf_counter() - t
    receivers_out = dict(spacings_m=[7, 15, 30], ms=round(1e3 * t_rx, 3),
                         Hz_abs=[float(abs(H[q, 2])) for q in range(3)],
                         Hz_background_abs=[float(abs(H[q, 2] - Ha[q, 2])) for q in range(3)])
    ref3 = os.path.join(ROOT, "tests", "golden", "config3_sample.npz")
    if os.path.exists(ref3):
        Hr = np.load(ref3)["H_total"]
        receivers_out["H_rel_err_vs_oracle"] = float(np.linalg.norm(H - Hr) / np.linalg.norm(Hr))
    log(f"receivers: {receivers_out}")

    large = None if args.no_large else matvec_large(ie, torch, ctx, s6, p)
    large_solve = None if args.no_large else solve_large(ie, torch, ctx, g, s6, p, acc)
    del x, Ea, E0
    small = None if args.no_small else config1_legs(ie, torch, args, acc)
    ex1 = None if args.no_ex1 else example1_bench(ie, torch, acc)
    batch = None if args.no_batch else batch_bench(ie, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, fp64_stats)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": round(total / args.steps, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"{LARGE_WORKLOAD}; plain float64 method: full-domain "
                               f"contraction-form GMRES({HEADLINE_RESTART}) from zero in complex128, "
                               "tol 1e-6",
                   "grid": list(p.n), "its": fp64_stats.its, "restarts": fp64_stats.restarts,
                   "relres": float(f"{fp64_stats.relres:.3e}"),
                   "matvecs64": fp64_stats.matvecs64,
                   "graph_cycles": fp64_stats.graph_cycles,
                   "green_setup_s": round(setup_s, 5),
                   "matvecs_per_s": round(fp64_stats.matvecs64 / (total / args.steps), 1)},
        "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic_bytes is None else int(traffic_bytes),
                     "traffic_source": traffic_src, "template": dom_kernel,
                     "avg_launch_ms": round(avg_ms, 5),
                     "launches": dom["launches"], "bytes_per_launch": int(dom["bytes_per_launch"]),
                     "share_of_profiled_time": round(dom["total_ms"] / prof_total, 3),
                     "measured": "HIP events on the launch stream around every launch, in a "
                                 "profiled replay of the timed step (direct launches)",
                     "rocprof": rocprof},
        "roofline_alu": pass_alu(dom, avg_ms),
        "cpu_baseline": cpu,
        "chosen_form": chosen,
        "induction_log": receivers_out,
        "matvec_large": large,
        "solve_large": large_solve,
        "config1": small,
        "example1": ex1,
        "batch": batch,
        "autotune_full_grid": {f"{r['precision']} {r['pass']}": r["variant"] for r in tuning
                               if r["grid"] == list(p.n)},
        "tuning_file": tuning_file,
        "accuracy": acc,
    }
    print(json.dumps(out))
    ie.ie_ctx_destroy(ctx)
    if args.save_tuning:
        ie.ie_tuning_save(args.save_tuning)


def config1_legs(ie, torch, args, acc):
    """The 64^3 three-layer dipping TI model (seed 101, 2 MHz): the chosen form, plain float64
    (full-domain GMRES(10) and (16), block GS with the adaptive inner tolerance), mixed block
    GS and Jacobi, the Krylov outer iteration over one GS sweep, the operator alone and the
    learned-guess comparison, with errors against the stored oracle field."""
    import synth
    p = synth.config1()
    nx, ny, nz = p.n
    zb = (0, nz // 2, nz)
    g = ie.make_grid(p.n, p.h, p.origin)
    ctx = ie.ie_green_setup(g, ie.ie_medium(p.sigma0, p.freq, 0.0), zb, ie.IE_FP64 | ie.IE_MIXED)
    s6 = torch.from_numpy(p.sigma6).cuda()
    shape = (3, nz, ny, nx)
    E = torch.zeros(shape, dtype=torch.complex128, device="cuda:0")
    Ea = torch.zeros_like(E)
    prob = dict(grid=g, sigma6=s6, sources=p.sources, E_total=E, E_anom=Ea)
    E0 = torch.zeros_like(E)
    ie.ie_background_field(ctx, p.sources, E0)
    ref = None
    refp = os.path.join(ROOT, "tests", "golden", "config1_Ea.npz")
    if os.path.exists(refp):
        ref = np.load(refp)["Ea"].astype(np.complex128)

    def err(a):
        return None if ref is None else float(np.linalg.norm(a - ref) / np.linalg.norm(ref))

    def solve_dd(opts):
        solve = lambda: ie.ie_dd_solve([ctx], [prob], opts)[1][0]  # noqa: E731
        solve()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = solve()
        torch.cuda.synchronize()
        return time.perf_counter() - t, st, Ea.cpu().numpy()

    def solve_full(precision, restart):
        x = torch.zeros_like(E0)

        def run():
            ie.ie_background_field(ctx, p.sources, E0)
            x.zero_()
            return ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, precision=precision, form=ie.IE_CIE,
                               restart=restart)[1]
        run()
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            gst = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), gst, (x - E0).cpu().numpy()

    out = {"workload": "64^3 cells of 0.25 m, three tilted-TI layers dipping 30 deg (seed 101), "
                       "2 MHz, z dipole; tol 1e-6"}
    t_c, st_c, Ea_c = solve_full(ie.IE_MIXED, CHOSEN_RESTART)
    out["chosen_full_mixed"] = dict(s=round(t_c, 5), its=st_c.its, Ea_rel_err=err(Ea_c))
    acc["config1_chosen_Ea_rel_err"] = err(Ea_c)
    receivers = None
    if not args.no_plain:
        t_f, st_f, Ea_f = solve_full(ie.IE_FP64, 10)
        t_r, st_r, _ = solve_full(ie.IE_FP64, CHOSEN_RESTART)
        out["fp64_full_gmres10"] = dict(s=round(t_f, 5), its=st_f.its, Ea_rel_err=err(Ea_f))
        out["fp64_full_gmres16"] = dict(s=round(t_r, 5), its=st_r.its)
        for name, scheme, prec, extra in (
                ("fp64_dd_gs_adaptive", ie.IE_GS, ie.IE_FP64, {}),
                ("mixed_dd_gs_adaptive", ie.IE_GS, ie.IE_MIXED, {}),
                ("mixed_dd_jacobi_adaptive", ie.IE_JACOBI, ie.IE_MIXED, {}),
                # inner tolerance 0.3: the fastest of 0.5 / 0.3 / 0.1 / 0.03 / 0.01 on this model
                ("mixed_fgmres_gs", ie.IE_FGMRES_GS, ie.IE_MIXED,
                 dict(inner_tol_fixed=0.3, init=ie.IE_INIT_ZERO, max_sweeps=120))):
            kw = dict(adaptive=True, tol=1e-6, precision=prec, form=ie.IE_CIE, restart=10)
            kw.update(extra)
            dt, st, Ea_d = solve_dd(ie.dd_opts(scheme=scheme, **kw))
            out[name] = dict(s=round(dt, 5), sweeps=st.sweeps, its=st.total_its,
                             Ea_rel_err=err(Ea_d))
        best = min(out["fp64_full_gmres10"]["s"], out["fp64_full_gmres16"]["s"],
                   out["fp64_dd_gs_adaptive"]["s"])
        out["plain_fp64_best_s"] = best
        out["speedup_chosen_vs_plain"] = round(best / t_c, 3)
    # operator alone (both precisions; the padded arrays of this grid fit the last-level cache)
    mv = {}
    tuning = ie.ie_ctx_tuning(ctx)
    for prec, dt_, nm in ((ie.IE_FP64, torch.complex128, "fp64"), (ie.IE_MIXED, torch.complex64,
                                                                    "c64")):
        xx = torch.randn(shape, dtype=dt_, device="cuda:0")
        yy = torch.empty_like(xx)
        ie.ie_matvec(ctx, s6, xx, yy, ie.IE_CIE, prec)
        torch.cuda.synchronize()
        ie.ie_profile_begin()
        reps = 20
        for _ in range(reps):
            ie.ie_matvec(ctx, s6, xx, yy, ie.IE_CIE, prec)
        pr = ie.ie_profile_end()
        passes = [k for k in pr if k["name"].split()[0] in PASSES]
        t_ms = sum(k["total_ms"] for k in passes) / reps
        byts = sum(k["bytes_per_launch"] * k["launches"] for k in passes) / reps
        tr = measured_traffic({k["name"]: k for k in passes}, tuning, p.n)
        mv[nm] = dict(ms=round(t_ms, 4), algorithmic_bytes=int(byts), cache_resident=True,
                      gbs=round(byts / (t_ms * 1e-3) / 1e9, 1),
                      traffic_bytes=None if tr is None else int(tr),
                      matvecs_per_s=round(1e3 / t_ms, 1),
                      passes_us={k["name"].split()[0]: round(1e3 * k["total_ms"] / k["launches"], 1)
                                 for k in passes})
    out["matvec"] = mv
    # one Arnoldi step of the chosen form: the chosen solve's time per iteration (restart work
    # included), and the algorithmic bytes of one step (operator, then the dots-and-norm pass
    # over j + 1 basis vectors and w and the update pass over j + 1 vectors, w read and written,
    # averaged over a restart cycle of CHOSEN_RESTART steps)
    vec = 3 * p.n[0] * p.n[1] * p.n[2] * 8.0
    gs = sum((j + 2) * vec + (j + 3) * vec for j in range(CHOSEN_RESTART)) / CHOSEN_RESTART
    step_bytes = mv["c64"]["algorithmic_bytes"] + gs
    step_us = 1e6 * t_c / st_c.its
    out["arnoldi_step"] = dict(us=round(step_us, 1), algorithmic_bytes=int(step_bytes),
                               gbs=round(step_bytes / (step_us * 1e-6) / 1e9, 1),
                               operator_us=round(1e3 * mv["c64"]["ms"], 1))
    if not args.no_nn:
        out["learned_guess"] = learned_bench(ie, torch, ctx, s6, p, ref)
    ie.ie_ctx_destroy(ctx)
    log(f"64^3 model: {out}")
    return out


def pass_alu(dom, avg_ms):
    """An operator pass against the vector-ALU peak, model flops per launch: 5 L log2 L per
    length-L transform (three components, forward and inverse in the x pass, one direction in the
    others) plus 72 per point for the tensor multiply of the x pass."""
    parts = dom["name"].split()
    if len(parts) < 3 or parts[0] not in ("xconv", "zfwd", "zinv") or not parts[2].startswith("L"):
        return None
    lx, ly, lz = (int(v) for v in parts[2][1:].split("x"))
    batch = int(parts[-1][1:]) if parts[-1].startswith("b") else 1
    nz = int(parts[3][2:]) if len(parts) > 3 and parts[3].startswith("nz") else lz // 2
    if parts[0] == "xconv":
        flops = float(ly * lz * batch) * (6 * 5 * lx * float(np.log2(lx)) + 72 * lx)
    else:  # a z pass over the columns of the (ny, nx) plane; ny, nx from LY, LX at 2x padding
        flops = float((ly // 2) * (lx // 2) * batch) * 3 * 5 * lz * float(np.log2(lz))
    tf = float(flops / (avg_ms * 1e-3) / 1e12)
    return {"bound": "alu", "achieved": round(tf, 2), "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tf / VALU_PEAK_TFLOPS, 4),
            "flops_per_launch": int(flops), "kernel": dom["name"]}


PASSES = ("zfwd", "yfwd", "xconv", "yinv", "zinv")
PASS_NAMES = {"zfwd": "k_zfwd", "zinv": "k_zinv", "xconv": "k_xconv", "yfwd": "k_colfft",
              "yinv": "k_colfft"}


def template_name(prof_name, tuning, grid):
    """Kernel template name (as rocprofv3 prints it) of a library profiler entry on the full
    grid, with the launch variant the autotuner chose, e.g. 'k_xconv2<double, 256, 0>'."""
    parts = prof_name.split()
    if len(parts) < 3 or parts[0] not in PASS_NAMES:
        return None
    prec = parts[1]
    m = [r for r in tuning if r["grid"] == list(grid) and r["precision"] == prec
         and r["pass"] == parts[0]]
    return m[0]["kernel"] if m else None


def measured_traffic(passes, tuning, grid):
    """HBM bytes of one operator application from the committed counter summaries (FETCH_SIZE +
    WRITE_SIZE per launch of each pass's chosen variant), or None if any pass has no entry for
    the current kernel sources."""
    from paper_2306_17537_amd import traffic
    tot = 0.0
    for k in passes.values():
        tn = template_name(k["name"], tuning, grid)
        hit = traffic.lookup(tn) if tn else None
        if hit is None:
            return None
        tot += hit[0]
    return tot


def rocprof_operator(passes, tuning, grid, byts):
    """One operator application timed as the sum of the rocprofv3 kernel-trace averages of its
    five passes (the chosen variants, from the committed trace of the timed solves: pure kernel
    time, no launch gaps), with its HBM fraction; None unless every pass has an entry for the
    current kernel sources."""
    from paper_2306_17537_amd import traffic
    us = 0.0
    for k in passes.values():
        tn = template_name(k["name"], tuning, grid)
        hit = traffic.trace_lookup(tn, summary=HEADLINE_TRACE) if tn else None
        if hit is None:
            return None
        us += hit[0]
    gbs = byts / (us * 1e-6) / 1e9
    return {"us": round(us, 1), "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "source": "profiles/" + HEADLINE_TRACE}


def solve_large(ie, torch, ctx, g, s6, p, acc):
    """The block forms on the 128x128x256 grid (four z slabs of 64), each from a zero start to
    e <= 1e-6: the Krylov outer iteration over one block GS or block Jacobi sweep (mixed, blocks
    to 0.3) and stationary block GS with the adaptive inner tolerance (Alg. 1, mixed)."""
    E = torch.zeros((3,) + tuple(reversed(p.n)), dtype=torch.complex128, device="cuda:0")
    Ea = torch.zeros_like(E)
    out = {"workload": f"{LARGE_WORKLOAD}; z slabs {list(p.z_bounds)}, tol 1e-6, zero start"}
    for name, scheme, sweeps in (("fgmres_gs_mixed", ie.IE_FGMRES_GS, 60),
                                 ("fgmres_jacobi_mixed", ie.IE_FGMRES_JACOBI, 60),
                                 ("dd_gs_a_mixed", ie.IE_GS, 20)):
        opts = ie.dd_opts(scheme=scheme, adaptive=scheme == ie.IE_GS, tol=1e-6,
                          inner_tol_fixed=0.3, init=ie.IE_INIT_ZERO, precision=ie.IE_MIXED,
                          form=ie.IE_CIE, restart=CHOSEN_RESTART, max_sweeps=sweeps, max_its=5000)

        def run(opts=opts):
            return ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=s6, sources=p.sources, E_total=E,
                                               E_anom=Ea)], opts, allow_noconv=True)
        run()  # warm-up: graphs, workspaces
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, st = run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = st[0]
        out[name] = dict(s=round(dt, 4), sweeps=st.sweeps, inner_its=st.total_its,
                         relres=float(f"{st.relres[st.sweeps]:.3e}"),
                         converged=bool(st.relres[st.sweeps] <= 1e-6), status=int(rc))
        if st.relres[st.sweeps] <= 1e-6:
            out[name]["Ea_rel_err"] = sample_error(Ea.cpu().numpy(), "config3")
            acc[f"large_{name}_Ea_rel_err"] = out[name]["Ea_rel_err"]
    del E, Ea
    log(f"solve large: {out}")
    return out


def matvec_large(ie, torch, ctx, s6, p):
    """The operator alone on the 128x128x256 grid: the working set of a padded three-component
    array exceeds the 256 MB last-level cache, so this is the HBM-bound case."""
    nx, ny, nz = p.n
    out = {}
    tuning = ie.ie_ctx_tuning(ctx)
    for prec, dt_, nm in ((ie.IE_MIXED, torch.complex64, "c64"), (ie.IE_FP64, torch.complex128, "fp64")):
        x = torch.randn((3, nz, ny, nx), dtype=dt_, device="cuda:0")
        y = torch.empty_like(x)
        ie.ie_matvec(ctx, s6, x, y, ie.IE_CIE, prec)
        torch.cuda.synchronize()
        ie.ie_profile_begin()
        reps = 10
        for _ in range(reps):
            ie.ie_matvec(ctx, s6, x, y, ie.IE_CIE, prec)
        pr = ie.ie_profile_end()
        passes = {k["name"].split()[0]: k for k in pr
                  if k["name"].split()[0] in PASSES}
        t_ms = sum(k["total_ms"] for k in passes.values()) / reps
        byts = sum(k["bytes_per_launch"] * k["launches"] for k in passes.values()) / reps
        tr = measured_traffic(passes, tuning, p.n)
        rp = rocprof_operator(passes, tuning, p.n, byts)
        out[nm] = dict(us=round(1e3 * t_ms, 1), algorithmic_bytes=int(byts), rocprof=rp,
                       cache_resident=False,
                       gbs=round(byts / (t_ms * 1e-3) / 1e9, 1),
                       frac=round(byts / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       traffic_bytes=None if tr is None else int(tr),
                       traffic_gbs=None if tr is None else round(tr / (t_ms * 1e-3) / 1e9, 1),
                       matvecs_per_s=round(1e3 / t_ms, 1),
                       passes_us={n: round(1e3 * k["total_ms"] / k["launches"], 1)
                                  for n, k in passes.items()})
        del x, y
    out["workload"] = f"{LARGE_WORKLOAD}; contraction-form operator, 10 launches"
    log(f"matvec large: {out}")
    return out


def example1_bench(ie, torch, acc):
    """The isolated sub-domains example (sec. 3.1) as the paper ran it: conventional form,
    float64, GMRES(10) to e = 1e-6, full domain vs block Gauss-Seidel with fixed inner tolerance
    over [background | anomaly | background | anomaly | background]; fields in the anomalies and
    the magnetic field at 20 receivers against the stored oracle reference."""
    import synth
    p = synth.example1()
    nx, ny, nz = p.n
    g = ie.make_grid(p.n, p.h, p.origin)
    ctx = ie.ie_green_setup(g, ie.ie_medium(p.sigma0, p.freq, 0.0), p.z_bounds, ie.IE_FP64)
    s6 = torch.from_numpy(p.sigma6).cuda()
    shape = (3, nz, ny, nx)
    E0 = torch.empty(shape, dtype=torch.complex128, device="cuda:0")
    out = {}
    refp = os.path.join(ROOT, "tests", "golden", "example1_sample.npz")
    try:
        for rep in range(2):  # the first pass warms up every kernel shape
            torch.cuda.synchronize()
            t = time.perf_counter()
            ie.ie_background_field(ctx, p.sources, E0)
            x = E0.clone()
            _, gst = ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, precision=ie.IE_FP64,
                                 form=ie.IE_CONVENTIONAL)
            torch.cuda.synchronize()
            t_full = time.perf_counter() - t
            Ed = torch.zeros(shape, dtype=torch.complex128, device="cuda:0")
            opts = ie.dd_opts(scheme=ie.IE_GS, adaptive=False, tol=1e-6, inner_tol_fixed=1e-6,
                              precision=ie.IE_FP64, form=ie.IE_CONVENTIONAL, max_sweeps=30)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=s6, sources=p.sources,
                                                E_total=Ed)], opts)
            torch.cuda.synchronize()
            t_dd = time.perf_counter() - t
            # the same with e over the anomalous cells only, as the paper computes it there
            Eda = torch.zeros(shape, dtype=torch.complex128, device="cuda:0")
            opts.residual_cells = ie.IE_RESID_ANOMALOUS
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, sta = ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=s6, sources=p.sources,
                                                 E_total=Eda)], opts)
            torch.cuda.synchronize()
            t_dda = time.perf_counter() - t
        out = dict(workload="128^3 cells of 0.25 m, two 0.01 S/m anomalies 30x30x7.5 m, 10 m "
                            "apart, 24 kHz x dipole; conventional form, float64, e <= 1e-6",
                   full_s=round(t_full, 4), full_its=int(gst.its), dd_gs_s=round(t_dd, 4),
                   dd_sweeps=int(st[0].sweeps), dd_inner_its=int(st[0].total_its),
                   dd_gs_anomalous_residual=dict(s=round(t_dda, 4), sweeps=int(sta[0].sweeps),
                                                 inner_its=int(sta[0].total_its)),
                   paper_context="MATLAB on a laptop GPU: full 53 s (86 its), DD-GS 23 s "
                                 "(4 sweeps, 278 its)")
        if os.path.exists(refp):
            d = np.load(refp)
            for name, E in (("full", x), ("dd_gs", Ed), ("dd_gs_anomalous_residual", Eda)):
                out[f"{name}_Ea_rel_err"] = sample_error((E - E0).cpu().numpy(), "example1")
                H, _ = ie.ie_receivers(ctx, s6, p.sources, E, d["rx"])
                out[f"{name}_H_rel_err"] = float(np.mean(
                    np.linalg.norm(H - d["H_total"], axis=1) /
                    np.linalg.norm(d["H_total"], axis=1)))
                acc[f"example1_{name}_Ea_rel_err"] = out[f"{name}_Ea_rel_err"]
    finally:
        ie.ie_ctx_destroy(ctx)
    log(f"example 1: {out}")
    return out


def learned_bench(ie, torch, ctx, s6, p, ref):
    """The same full-domain mixed solve from a zero start and from the trained network's guess
    (judged by one zero-start restart cycle; both judge cycles counted)."""
    from paper_2306_17537_amd import guess
    nn = guess.create()
    nx, ny, nz = p.n
    E0 = torch.empty((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0")
    out = {}
    try:
        for name in ("zero", "learned"):
            ts, its, used = [], 0, 0
            for _ in range(3):
                x = torch.zeros_like(E0)
                torch.cuda.synchronize()
                t = time.perf_counter()
                ie.ie_background_field(ctx, p.sources, E0)
                if name == "learned":
                    used = guess.solve_learned_start(ctx, nn, s6, E0, x, restart=CHOSEN_RESTART)
                _, st = ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, precision=ie.IE_MIXED,
                                    form=ie.IE_CIE, restart=CHOSEN_RESTART)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
                its = st.its + (2 * CHOSEN_RESTART if name == "learned" else 0)
            err = None
            if ref is not None:
                err = float(np.linalg.norm((x - E0).cpu().numpy() - ref) / np.linalg.norm(ref))
            out[name] = dict(s=round(float(np.median(ts)), 5), its=int(its), Ea_rel_err=err)
            if name == "learned":
                out[name]["learned_start_won_judge"] = int(used)
        out["gemm_roofline"] = nn_gemm_roofline(ie, torch, ctx, nn, s6, E0)
    finally:
        ie.ie_nn_destroy(nn)
    out["network"] = "3-D encoder-decoder, 4 levels, base 32 channels, BF16 MFMA (weights in " \
                     "paper_2306_17537_amd/weights, trained on 2000 solver-generated 32^3 blocks)"
    out["gain"] = round(out["zero"]["s"] / out["learned"]["s"], 3)
    log(f"learned guess: {out}")
    return out


def nn_gemm_roofline(ie, torch, ctx, nn, s6, E0):
    """The network's convolutions (BF16 16x16x32 MFMA; implicit GEMMs where the channel counts
    allow, else im2col + GEMM) in one inference on the 64^3 model, timed with HIP events per
    launch: dense flops (2 M N K per launch) per second against the 2.5 PFLOP/s dense BF16 peak,
    and the share of the inference spent in im2col."""
    from paper_2306_17537_amd import guess
    x = torch.zeros_like(E0)
    ie.ie_profile_begin()
    guess.solve_learned_start(ctx, nn, s6, E0, x, restart=CHOSEN_RESTART)
    prof = ie.ie_profile_end()
    gem = [k for k in prof if k["name"].startswith(("nn_gemm", "nn_conv"))]
    if not gem:
        return None
    flops = 0.0
    for k in gem:
        m = re.search(r"M(\d+)xN(\d+)xK(\d+)", k["name"])
        flops += 2.0 * int(m.group(1)) * int(m.group(2)) * int(m.group(3)) * k["launches"]
    t = sum(k["total_ms"] for k in gem) * 1e-3
    nn_t = sum(k["total_ms"] for k in prof if k["name"].startswith("nn_")) * 1e-3
    im2col = sum(k["total_ms"] for k in prof if k["name"].startswith("nn_im2col")) * 1e-3
    byts = sum(k["bytes_per_launch"] * k["launches"] for k in gem)
    big = max(gem, key=lambda k: k["total_ms"])
    # bytes: the operands as read from memory (the activations once for an implicit GEMM, the
    # materialised M x 27 C_in matrix otherwise), weights and output
    return {"bound": "mfma", "achieved": round(flops / t / 1e12, 2), "peak": 2500.0,
            "unit": "TFLOP/s", "frac": round(flops / t / 1e12 / 2500.0, 4),
            "flop_per_byte": round(flops / byts, 1),
            "hbm_achieved_gbs": round(byts / t / 1e9, 1),
            "hbm_frac": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
            "gemm_launches": sum(k["launches"] for k in gem), "gemm_ms": round(1e3 * t, 3),
            "largest": big["name"], "im2col_share_of_network": round(im2col / nn_t, 3)}


def batch_bench(ie, torch):
    """Logging run: 64 tool positions x 2 frequencies = 128 solves on tool-centred grids of
    three shapes, one block each (full-domain mixed GMRES), all in ONE ie_dd_solve call;
    problems sharing (shape, frequency) are advanced as one batch (blockIdx.z).  Run with the
    default FFT lengths (3 * 2^k where shorter than the power of two) and again with powers of
    two only."""
    import dataclasses
    import synth
    args = parse()
    probs = [dataclasses.replace(p, z_bounds=(0, p.n[2])) for p in synth.config2()]
    opts = ie.dd_opts(tol=1e-6, adaptive=False, inner_tol_fixed=5e-7, precision=ie.IE_MIXED,
                      max_its=5000, restart=CHOSEN_RESTART)

    def build(pow2):
        ctxs, grids = {}, {}
        ie.ie_set_option(ie.IE_OPT_FFT_LENGTHS, pow2)
        try:
            t0 = time.perf_counter()
            for p in probs:
                key = (p.n, p.freq)
                if key not in ctxs:
                    g = ie.make_grid(p.n, p.h, p.origin)
                    ctxs[key] = ie.ie_green_setup(g, ie.ie_medium(p.sigma0, p.freq, 0.0),
                                                  p.z_bounds)
                    grids[key] = g
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
        finally:
            ie.ie_set_option(ie.IE_OPT_FFT_LENGTHS, 0)
        data = []
        for p in probs:
            key = (p.n, p.freq)
            E = torch.zeros((3, p.n[2], p.n[1], p.n[0]), dtype=torch.complex128,
                            device="cuda:0")
            data.append((ctxs[key], dict(grid=grids[key],
                                         sigma6=torch.from_numpy(p.sigma6).cuda(),
                                         sources=p.sources, E_total=E)))
        lengths = sorted({(k[0], tuple(ie.ie_ctx_tuning(c)[0]["fft"])) for k, c in ctxs.items()})
        return ctxs, data, t_setup, {f"{n[0]}x{n[1]}x{n[2]}": list(L) for n, L in lengths}

    def run(data, sel):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = ie.ie_dd_solve([data[i][0] for i in sel], [data[i][1] for i in sel], opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t, st

    allsel = list(range(len(probs)))
    ctxs, data, t_setup, lengths = build(0)
    run(data, allsel[:12])  # warm-up of every kernel shape
    log("logging run: 128 solves in one call")
    t_all, st = run(data, allsel)
    mv = sum(s.matvecs32 + s.matvecs64 for s in st)
    worst = max(s.relres[s.sweeps] for s in st)
    nseq = min(args.batch_seq, len(probs))
    t_seq = sum(run(data, [i])[0] for i in range(nseq))
    t_bat, _ = run(data, list(range(nseq)))
    for c in ctxs.values():
        ie.ie_ctx_destroy(c)
    del data
    log("logging run: powers-of-two FFT lengths")
    ctxs2, data2, t_setup2, lengths2 = build(1)
    run(data2, allsel[:12])
    t_all2, st2 = run(data2, allsel)
    mv2 = sum(s.matvecs32 + s.matvecs64 for s in st2)
    for c in ctxs2.values():
        ie.ie_ctx_destroy(c)
    del data2
    out = dict(workload="config2: 64 positions x {400 kHz, 2 MHz} = 128 solves, grids "
                        "32^3 / 48x48x64 / 64x64x96 (seed 202), full-domain mixed "
                        f"GMRES({CHOSEN_RESTART}), "
                        "tol 1e-6, one ie_dd_solve call",
               solves=len(probs), groups=len(ctxs), wall_s=round(t_all, 4),
               solves_per_s=round(len(probs) / t_all, 2), matvecs=mv,
               matvecs_per_s=round(mv / t_all, 1), worst_relres=worst,
               green_setup_s=round(t_setup, 3), fft_lengths=lengths,
               subset=dict(problems=nseq, one_call_each_s=round(t_seq, 4),
                           batched_s=round(t_bat, 4), speedup=round(t_seq / t_bat, 3)),
               pow2_lengths=dict(fft_lengths=lengths2, wall_s=round(t_all2, 4),
                                 solves_per_s=round(len(probs) / t_all2, 2), matvecs=mv2,
                                 worst_relres=max(s.relres[s.sweeps] for s in st2),
                                 green_setup_s=round(t_setup2, 3),
                                 speedup_of_default=round(t_all2 / t_all, 3)))
    log(f"batch: {out}")
    return out


def cpu_baseline(p, gst):
    """The oracle on this host: its full-domain contraction-form solve of the same problem in
    float64 (scipy FFTs and BLAS on every host core), timed over a bounded sample of restarted
    GMRES iterations and scaled to one solve with the operator-application count of the GPU run."""
    import scipy.fft
    from threadpoolctl import threadpool_limits
    from oracle import operator, solve as osolve
    from oracle.gmres import gmres
    cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    with scipy.fft.set_workers(cores), threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        st = osolve.setup(p)
        t_setup = time.perf_counter() - t0
        b, a, _ = operator.cie_tensors(st.dsig, p.sigma0)
        rhs = np.sqrt(p.sigma0) * st.E0
        its = 4
        t0 = time.perf_counter()
        _, info = gmres(lambda v: operator.apply_C(st.Ghat, b, v, p.sigma0, st.n), rhs, None,
                        1e-14, HEADLINE_RESTART, its)
        t_sample = time.perf_counter() - t0
        # one iteration = one operator application, plus the true residual at the end
        napp = info["its"] + info["restarts"] + 1
        t_app = t_sample / napp
    napp_gpu = gst.its + gst.restarts + 1
    est = napp_gpu * t_app
    return {"value": round(est, 2), "unit": "s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "threads": {"scipy_fft_workers": cores, "blas": cores},
            "sample": f"oracle float64 full-domain contraction-form GMRES({HEADLINE_RESTART}) of the "
                      f"same 128x128x256 problem on this host: {info['its']} iterations from zero "
                      f"({napp} operator applications, {t_sample:.2f} s, {t_app:.3f} s each), "
                      f"scaled to the GPU solve's {napp_gpu} applications ({gst.its} iterations, "
                      f"{gst.restarts + 1} restarts); oracle setup {t_setup:.1f} s excluded like "
                      "the GPU setup"}


if __name__ == "__main__":
    main()
