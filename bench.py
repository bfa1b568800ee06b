#!/usr/bin/env python3
"""Benchmark of the integral-equation solver on one MI355X.

Workload (one "step"): one complete solve of the 64^3 three-layer dipping TI model (cell
0.25 m, 2 MHz, z dipole at the centre) to full-domain relative residual 1e-6 (eq. 9) by the
chosen form: background field, contrast preparation and restarted GMRES(12) from a zero start
on the contraction form in mixed precision (complex64 Krylov vectors and convolutions; float64
residual at every restart, Arnoldi scalars, Givens rotations and solution accumulation).  The Green's spectrum is
built once before the timed region (it depends on grid and medium only) and timed separately.
The same solve by Alg. 1 (block Gauss-Seidel and Jacobi over two z slabs, float64 and mixed)
and by plain float64 GMRES is timed in the same run and reported beside it.

Printed: one JSON line with the contract fields plus
  roofline     - dominant kernel of the timed region: algorithmic bytes / duration, HIP events
                 on the launch stream (library launch profiler), against 8 TB/s;
  roofline_alu - the same kernel against the non-packed vector-ALU peak (model flops: 5 L log2 L
                 per transform, 72 per point for the tensor multiply);
  cpu_baseline - the CPU oracle on this host, sampled and scaled to one solve;
  plain_fp64   - the same solve in plain float64 (best of full-domain GMRES(10), GMRES(16) and
                 DD-GS-A);
  solve_large  - the chosen form, plain float64 and two DD forms on the 128x128x256 grid;
  accuracy     - relative L2 error of the anomalous field against the stored oracle reference.
"""
import argparse
import json
import os
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
# Restart length of the chosen form.  The paper runs GMRES(10).  In mixed precision, summed over
# this model and four held-out seeds of it, restart 16 took 6 % less time than 10 and 2 % less
# than 12 (fewer restarts, each a float64 residual; fewer Arnoldi steps).  Plain float64 is
# timed at 10 and at this length.
CHOSEN_RESTART = 16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-seq", type=int, default=16,
                    help="problems of the logging run also solved one call each (speed-up)")
    ap.add_argument("--profile-json", default=None, help="write the kernel profile here")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="first run the 1 GiB fill and copy kernels that scale the HBM counters")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the operator and the solves on the 128x128x256 grid")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned-guess comparison")
    ap.add_argument("--no-ex1", action="store_true",
                    help="skip the isolated sub-domains example (128^3, DD vs full domain)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
    if args.pmc_calibration:
        from paper_2306_17537_amd import traffic
        traffic.calibrate()
    p = synth.config1()
    nx, ny, nz = p.n
    zb = (0, nz // 2, nz)
    g = ie.make_grid(p.n, p.h, p.origin)
    med = ie.ie_medium(p.sigma0, p.freq, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = ie.ie_green_setup(g, med, zb, ie.IE_FP64 | ie.IE_MIXED)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"green setup {setup_s * 1e3:.1f} ms")
    s6 = torch.from_numpy(p.sigma6).cuda()
    shape = (3, nz, ny, nx)
    E = torch.zeros(shape, dtype=torch.complex128, device="cuda:0")
    Ea = torch.zeros_like(E)
    prob = dict(grid=g, sigma6=s6, sources=p.sources, E_total=E, E_anom=Ea)

    chosen = ie.dd_opts(scheme=ie.IE_GS, adaptive=True, tol=1e-6, precision=ie.IE_MIXED,
                        form=ie.IE_CIE, restart=10)

    def solve_dd(opts):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = ie.ie_dd_solve([ctx], [prob], opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t, st[0]

    E0 = torch.zeros_like(E)
    ie.ie_background_field(ctx, p.sources, E0)

    def solve_full(precision, restart=10):
        x = torch.zeros_like(E0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, gst = ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, precision=precision, form=ie.IE_CIE,
                             restart=restart)
        torch.cuda.synchronize()
        return time.perf_counter() - t, gst, (x - E0).cpu().numpy()

    def solve_chosen():
        # background field + contrast + mixed-precision GMRES from a zero start, all inside the
        # timed step
        torch.cuda.synchronize()
        t = time.perf_counter()
        ie.ie_background_field(ctx, p.sources, E0)
        x = torch.zeros_like(E0)
        _, gst = ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, precision=ie.IE_MIXED, form=ie.IE_CIE,
                             restart=CHOSEN_RESTART)
        torch.sub(x, E0, out=Ea)
        torch.cuda.synchronize()
        return time.perf_counter() - t, gst

    for _ in range(args.warmup):
        solve_chosen()
    log("timed region")
    times = []
    for _ in range(args.steps):
        dt, st = solve_chosen()
        times.append(dt)
    total = sum(times)
    ms_per_step = 1e3 * total / args.steps
    chosen_stats = st
    Ea_chosen = Ea.cpu().numpy()
    log(f"chosen form: {ms_per_step:.2f} ms/solve, its={st.its} refinements={st.refinements} "
        f"mv32={st.matvecs32} mv64={st.matvecs64} graph_cycles={st.graph_cycles}")

    # the paper's observable: H at receivers 7, 15 and 30 m above the transmitter (eqs. 4, 6)
    rx = [[0.0, 0.0, 7.0], [0.0, 0.0, 15.0], [0.0, 0.0, 30.0]]
    Et = Ea + E0
    torch.cuda.synchronize()
    t = time.perf_counter()
    H, Ha = ie.ie_receivers(ctx, s6, p.sources, Et, rx)
    t_rx = time.perf_counter() - t
    receivers_out = dict(spacings_m=[7, 15, 30], ms=round(1e3 * t_rx, 3),
                         Hz_abs=[float(abs(H[q, 2])) for q in range(3)],
                         Hz_background_abs=[float(abs(H[q, 2] - Ha[q, 2])) for q in range(3)])
    log(f"receivers: {receivers_out}")

    # the same steps with direct kernel launches (no graph replay), then profiled
    ie.ie_set_option(ie.IE_OPT_GRAPHS, 0)
    t_eager = [solve_chosen()[0] for _ in range(args.steps)]
    ie.ie_set_option(ie.IE_OPT_GRAPHS, 1)
    ie.ie_profile_begin()
    t_prof = [solve_chosen()[0] for _ in range(args.steps)]
    prof = ie.ie_profile_end()
    log(f"direct launches: {1e3 * sum(t_eager) / args.steps:.2f} ms/solve; profiled "
        f"{1e3 * sum(t_prof) / args.steps:.2f} ms/solve")

    # dominant kernel (largest share of the profiled replay of the timed steps)
    kern = [k for k in prof if not k["name"].startswith("finalise")]
    dom = kern[0]
    avg_ms = dom["total_ms"] / dom["launches"]
    achieved = dom["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    tuning = ie.ie_ctx_tuning(ctx)
    dom_kernel, traffic_bytes, traffic_src = template_name(dom["name"], tuning, p.n), None, None
    if dom_kernel:
        from paper_2306_17537_amd import traffic
        hit = traffic.lookup(dom_kernel)
        if hit is not None:
            traffic_bytes, _, traffic_src = hit[0], hit[1], os.path.relpath(hit[2], ROOT)
    prof_total = sum(k["total_ms"] for k in prof)
    if args.profile_json:
        with open(args.profile_json, "w") as f:
            json.dump(dict(kernels=prof, steps=args.steps), f, indent=1)

    # matvec throughput on the full grid (standalone, float64 and complex64)
    mv = {}
    for prec, dt_, nm in ((ie.IE_FP64, torch.complex128, "fp64"), (ie.IE_MIXED, torch.complex64, "c64")):
        x = torch.randn(shape, dtype=dt_, device="cuda:0")
        y = torch.empty_like(x)
        ie.ie_matvec(ctx, s6, x, y, ie.IE_CIE, prec)
        torch.cuda.synchronize()
        ie.ie_profile_begin()
        reps = 20
        for _ in range(reps):
            ie.ie_matvec(ctx, s6, x, y, ie.IE_CIE, prec)
        pr = ie.ie_profile_end()
        passes = [k for k in pr if k["name"].split()[0] in ("xfwd", "yfwd", "zconv", "yinv", "xinv")]
        t_ms = sum(k["total_ms"] for k in passes) / reps
        byts = sum(k["bytes_per_launch"] * k["launches"] for k in passes) / reps
        tr = measured_traffic({k["name"]: k for k in passes}, tuning, p.n)
        mv[nm] = dict(ms=round(t_ms, 4), algorithmic_bytes=int(byts),
                      cache_resident=True,  # padded arrays far below the 256 MB last-level cache
                      gbs=round(byts / (t_ms * 1e-3) / 1e9, 1),
                      traffic_bytes=None if tr is None else int(tr),
                      traffic_gbs=None if tr is None else round(tr / (t_ms * 1e-3) / 1e9, 1),
                      matvecs_per_s=round(1e3 / t_ms, 1))
    log(f"matvec: {mv}")
    large = None if args.no_large else matvec_large(ie, torch)
    large_solve = None if args.no_large else solve_large(ie, torch)

    # other forms on the same GPU: plain float64 (the better of full-domain GMRES and DD-GS-A),
    # full-domain mixed GMRES and mixed DD-Jacobi
    plain = None
    variants = {}
    acc = {}
    ref = None
    refp = os.path.join(ROOT, "tests", "golden", "config1_Ea.npz")
    if os.path.exists(refp):
        ref = np.load(refp)["Ea"].astype(np.complex128)
        rn = np.linalg.norm(ref)
        acc["chosen_Ea_rel_err"] = float(np.linalg.norm(Ea_chosen - ref) / rn)
    st_dd = None
    if not args.no_plain:
        fp64_dd = ie.dd_opts(scheme=ie.IE_GS, adaptive=True, tol=1e-6, precision=ie.IE_FP64,
                             form=ie.IE_CIE, restart=10)
        solve_dd(fp64_dd)
        t_dd, st_dd = solve_dd(fp64_dd)
        Ea_dd = Ea.cpu().numpy()
        solve_full(ie.IE_FP64)
        t_full, gst, Ea_full = solve_full(ie.IE_FP64)
        solve_full(ie.IE_FP64, CHOSEN_RESTART)
        t_full_r, gst_r, _ = solve_full(ie.IE_FP64, CHOSEN_RESTART)
        solve_dd(chosen)
        t_gm, st_gm = solve_dd(chosen)
        Ea_gm = Ea.cpu().numpy()
        jac = ie.dd_opts(scheme=ie.IE_JACOBI, adaptive=True, tol=1e-6, precision=ie.IE_MIXED,
                         form=ie.IE_CIE, restart=10)
        solve_dd(jac)
        t_j, st_j = solve_dd(jac)
        Ea_j = Ea.cpu().numpy()
        # Krylov outer iteration over the GS sweep (inner tolerance 0.3: the fastest of
        # 0.5 / 0.3 / 0.1 / 0.03 / 0.01 measured on this model)
        fg = ie.dd_opts(scheme=ie.IE_FGMRES_GS, tol=1e-6, inner_tol_fixed=0.3,
                        init=ie.IE_INIT_ZERO, precision=ie.IE_MIXED, form=ie.IE_CIE, restart=10,
                        max_sweeps=120)
        solve_dd(fg)
        t_fg, st_fg = solve_dd(fg)
        Ea_fg = Ea.cpu().numpy()
        plain = dict(dd_gs_a_fp64_s=round(t_dd, 5), dd_sweeps=st_dd.sweeps, dd_its=st_dd.total_its,
                     full_gmres_fp64_s=round(t_full, 5), full_its=gst.its,
                     full_gmres_chosen_restart_fp64_s=round(t_full_r, 5),
                     full_chosen_restart_its=gst_r.its,
                     best_s=round(min(t_dd, t_full, t_full_r), 5),
                     speedup_chosen_vs_plain=round(min(t_dd, t_full, t_full_r) /
                                                   (total / args.steps), 3))
        variants = dict(dd_gs_a_mixed_s=round(t_gm, 5), gs_mixed_sweeps=st_gm.sweeps,
                        gs_mixed_its=st_gm.total_its,
                        dd_jacobi_a_mixed_s=round(t_j, 5), jacobi_sweeps=st_j.sweeps,
                        jacobi_its=st_j.total_its, jacobi_blocks_batched=2,
                        fgmres_gs_mixed_s=round(t_fg, 5), fgmres_outer=st_fg.sweeps,
                        fgmres_inner_its=st_fg.total_its,
                        chosen_direct_launch_s=round(sum(t_eager) / args.steps, 5))
        if ref is not None:
            acc["plain_dd_Ea_rel_err"] = float(np.linalg.norm(Ea_dd - ref) / rn)
            acc["plain_full_Ea_rel_err"] = float(np.linalg.norm(Ea_full - ref) / rn)
            acc["dd_gs_mixed_Ea_rel_err"] = float(np.linalg.norm(Ea_gm - ref) / rn)
            acc["jacobi_mixed_Ea_rel_err"] = float(np.linalg.norm(Ea_j - ref) / rn)
            acc["fgmres_gs_mixed_Ea_rel_err"] = float(np.linalg.norm(Ea_fg - ref) / rn)
        log(f"plain fp64: {plain}")
        log(f"variants: {variants}")

    learned = None if args.no_nn else learned_bench(ie, torch, ctx, s6, p, ref)
    ex1 = None if args.no_ex1 else example1_bench(ie, torch)
    batch = None if args.no_batch else batch_bench(ie, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, chosen_stats)
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
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": "config1: 64^3 cells of 0.25 m, 3-layer TI dipping 30 deg "
                               "(seed 101), 2 MHz, z dipole; full-domain contraction-form "
                               f"GMRES({CHOSEN_RESTART}) from zero, complex64 Krylov/"
                               "convolutions + float64 restarts, tol 1e-6",
                   "grid": list(p.n), "its": chosen_stats.its,
                   "refinements": chosen_stats.refinements, "matvecs32": chosen_stats.matvecs32,
                   "matvecs64": chosen_stats.matvecs64, "graph_cycles": chosen_stats.graph_cycles,
                   "green_setup_s": round(setup_s, 5), "solves_per_s": round(args.steps / total, 3)},
        "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic_bytes is None else int(traffic_bytes),
                     "traffic_source": traffic_src, "template": dom_kernel,
                     "avg_launch_ms": round(avg_ms, 5),
                     "launches": dom["launches"], "bytes_per_launch": int(dom["bytes_per_launch"]),
                     "share_of_profiled_time": round(dom["total_ms"] / prof_total, 3),
                     "measured": "HIP events on the launch stream around every launch, in a "
                                 "profiled replay of the timed steps (direct launches)"},
        "roofline_alu": zconv_alu(dom, avg_ms),
        "cpu_baseline": cpu,
        "plain_fp64": plain,
        "variants": variants,
        "induction_log": receivers_out,
        "learned_guess": learned,
        "example1": ex1,
        "batch": batch,
        "matvec": mv,
        "matvec_large": large,
        "solve_large": large_solve,
        "autotune_full_grid": {f"{r['precision']} {r['pass']}": r["variant"] for r in tuning
                               if r["grid"] == list(p.n)},
        "accuracy": acc,
    }
    print(json.dumps(out))
    ie.ie_ctx_destroy(ctx)


def zconv_alu(dom, avg_ms):
    """The dominant kernel (the z pass) against the vector-ALU peak: model flops per launch =
    lines x (6 transforms x 5 L log2 L + 72 L) for L = LZ (three components, forward and
    inverse, unpruned) plus the 3x3 complex tensor multiply (72 flop per padded point)."""
    parts = dom["name"].split()
    if len(parts) < 3 or parts[0] != "zconv" or not parts[2].startswith("L"):
        return None
    lx, ly, lz = (int(v) for v in parts[2][1:].split("x"))
    batch = int(parts[-1][1:]) if parts[-1].startswith("b") else 1
    flops = float(lx * ly * batch) * (6 * 5 * lz * float(np.log2(lz)) + 72 * lz)
    tf = float(flops / (avg_ms * 1e-3) / 1e12)
    return {"bound": "alu", "achieved": round(tf, 2), "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tf / VALU_PEAK_TFLOPS, 4),
            "flops_per_launch": int(flops), "kernel": dom["name"]}


PASS_NAMES = {"xfwd": "k_xfwd", "xinv": "k_xinv", "zconv": "k_zconv", "yfwd": "k_colfft",
              "yinv": "k_colfft"}


def template_name(prof_name, tuning, grid):
    """Kernel template name (as rocprofv3 prints it) of a library profiler entry on the full
    grid, with the launch variant the autotuner chose, e.g. 'k_zconv<float, 128, 1>'."""
    parts = prof_name.split()
    if len(parts) < 3 or parts[0] not in PASS_NAMES:
        return None
    prec = parts[1]
    m = [r for r in tuning if r["grid"] == list(grid) and r["precision"] == prec
         and r["pass"] == parts[0]]
    if not m:
        return None
    t = "float" if prec == "c64" else "double"
    dims = parts[2][1:].split("x")
    if parts[0] in ("yfwd", "yinv"):
        L = int(dims[0])
        inv = "true" if parts[0] == "yinv" else "false"
        return f"k_colfft<{t}, {L}, {inv}, {m[0]['variant']}>"
    L = int(dims[2]) if parts[0] == "zconv" else int(dims[0])
    return f"{PASS_NAMES[parts[0]]}<{t}, {L}, {m[0]['variant']}>"


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


def solve_large(ie, torch):
    """Time to e <= 1e-6 on the 128x128x256 grid (six layers dipping 20 deg, principal values in
    [0.1, 10] S/m, 2 MHz, four z slabs of 64): full-domain contraction-form GMRES in mixed
    precision (the chosen form) and in plain float64, the Krylov outer iteration over one block
    GS or block Jacobi sweep (mixed, blocks to 0.3), and stationary block GS with the adaptive
    inner tolerance (Alg. 1, mixed, 20 sweeps), each from a zero start."""
    import synth
    p = synth.config3()
    nx, ny, nz = p.n
    g = ie.make_grid(p.n, p.h, p.origin)
    ctx = ie.ie_green_setup(g, ie.ie_medium(p.sigma0, p.freq, 0.0), p.z_bounds)
    s6 = torch.from_numpy(p.sigma6).cuda()
    E0 = torch.zeros((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0")
    ie.ie_background_field(ctx, p.sources, E0)
    out = {"workload": "config3 grid 128x128x256 (seed 303), 2 MHz, z slabs "
                       f"{list(p.z_bounds)}, tol 1e-6, zero start"}

    def timed(fn):
        fn()  # warm-up: graphs, workspaces
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    for name, prec, m in (("full_mixed", ie.IE_MIXED, CHOSEN_RESTART),
                          ("full_fp64", ie.IE_FP64, CHOSEN_RESTART),
                          ("full_fp64_gmres10", ie.IE_FP64, 10)):
        x = torch.zeros_like(E0)

        def run(x=x, prec=prec, m=m):
            x.zero_()
            return ie.ie_gmres(ctx, s6, E0, x, tol=1e-6, restart=m, precision=prec,
                               form=ie.IE_CIE, max_its=5000, allow_noconv=True)[1]
        dt, st = timed(run)
        out[name] = dict(s=round(dt, 4), its=st.its, relres=float(f"{st.relres:.3e}"))
        del x
    E = torch.zeros_like(E0)
    for name, scheme, sweeps in (("fgmres_gs_mixed", ie.IE_FGMRES_GS, 60),
                                 ("fgmres_jacobi_mixed", ie.IE_FGMRES_JACOBI, 60),
                                 ("dd_gs_a_mixed", ie.IE_GS, 20)):
        opts = ie.dd_opts(scheme=scheme, adaptive=scheme == ie.IE_GS, tol=1e-6,
                          inner_tol_fixed=0.3, init=ie.IE_INIT_ZERO, precision=ie.IE_MIXED,
                          form=ie.IE_CIE, restart=CHOSEN_RESTART, max_sweeps=sweeps, max_its=5000)

        def run(opts=opts):
            return ie.ie_dd_solve([ctx], [dict(grid=g, sigma6=s6, sources=p.sources, E_total=E)],
                                  opts, allow_noconv=True)[1][0]
        dt, st = timed(run)
        out[name] = dict(s=round(dt, 4), sweeps=st.sweeps, inner_its=st.total_its,
                         relres=float(f"{st.relres[st.sweeps]:.3e}"),
                         converged=bool(st.relres[st.sweeps] <= 1e-6))
    out["speedup_chosen_vs_plain"] = round(
        min(out["full_fp64"]["s"], out["full_fp64_gmres10"]["s"]) / out["full_mixed"]["s"], 3)
    del E, E0, s6
    ie.ie_ctx_destroy(ctx)
    log(f"solve large: {out}")
    return out


def matvec_large(ie, torch):
    """The operator on the 128x128x256 grid (6-layer model, 2 MHz): the working set of a padded
    three-component array exceeds the 256 MB last-level cache, so this is the HBM-bound case."""
    import synth
    p = synth.config3()
    nx, ny, nz = p.n
    g = ie.make_grid(p.n, p.h, p.origin)
    ctx = ie.ie_green_setup(g, ie.ie_medium(p.sigma0, p.freq, 0.0), None, ie.IE_FP64 | ie.IE_MIXED)
    s6 = torch.from_numpy(p.sigma6).cuda()
    out = {}
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
                  if k["name"].split()[0] in ("xfwd", "yfwd", "zconv", "yinv", "xinv")}
        t_ms = sum(k["total_ms"] for k in passes.values()) / reps
        byts = sum(k["bytes_per_launch"] * k["launches"] for k in passes.values()) / reps
        tr = measured_traffic(passes, ie.ie_ctx_tuning(ctx), p.n)
        out[nm] = dict(us=round(1e3 * t_ms, 1), algorithmic_bytes=int(byts),
                       cache_resident=False,
                       gbs=round(byts / (t_ms * 1e-3) / 1e9, 1),
                       frac=round(byts / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       traffic_bytes=None if tr is None else int(tr),
                       traffic_gbs=None if tr is None else round(tr / (t_ms * 1e-3) / 1e9, 1),
                       passes_us={n: round(1e3 * k["total_ms"] / k["launches"], 1)
                                  for n, k in passes.items()})
        del x, y
    ie.ie_ctx_destroy(ctx)
    out["workload"] = "config3 grid 128x128x256 (seed 303), contraction-form operator, 10 launches"
    log(f"matvec large: {out}")
    return out


def example1_bench(ie, torch):
    """The isolated sub-domains example (sec. 3.1) as the paper ran it: conventional form,
    float64, GMRES(10) to e = 1e-6, full domain vs block Gauss-Seidel with fixed inner tolerance
    over [background | anomaly | background | anomaly | background]."""
    import synth
    p = synth.example1()
    nx, ny, nz = p.n
    g = ie.make_grid(p.n, p.h, p.origin)
    ctx = ie.ie_green_setup(g, ie.ie_medium(p.sigma0, p.freq, 0.0), p.z_bounds, ie.IE_FP64)
    s6 = torch.from_numpy(p.sigma6).cuda()
    shape = (3, nz, ny, nx)
    E0 = torch.empty(shape, dtype=torch.complex128, device="cuda:0")
    out = {}
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
        out = dict(workload="128^3 cells of 0.25 m, two 0.01 S/m anomalies 30x30x7.5 m, 10 m "
                            "apart, 24 kHz x dipole; conventional form, float64, e <= 1e-6",
                   full_s=round(t_full, 4), full_its=int(gst.its), dd_gs_s=round(t_dd, 4),
                   dd_sweeps=int(st[0].sweeps), dd_inner_its=int(st[0].total_its),
                   paper_context="MATLAB on a laptop GPU: full 53 s (86 its), DD-GS 23 s "
                                 "(4 sweeps, 278 its)")
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
    finally:
        ie.ie_nn_destroy(nn)
    out["network"] = "3-D encoder-decoder, 4 levels, base 32 channels, BF16 MFMA (weights in " \
                     "paper_2306_17537_amd/weights, trained on 2000 solver-generated 32^3 blocks)"
    out["gain"] = round(out["zero"]["s"] / out["learned"]["s"], 3)
    log(f"learned guess: {out}")
    return out


def batch_bench(ie, torch):
    """Logging run: 64 tool positions x 2 frequencies = 128 solves on tool-centred grids of
    three shapes, one block each (full-domain mixed GMRES), all in ONE ie_dd_solve call;
    problems sharing (shape, frequency) are advanced as one batch (blockIdx.z)."""
    import dataclasses
    import synth
    args = parse()
    probs = [dataclasses.replace(p, z_bounds=(0, p.n[2])) for p in synth.config2()]
    ctxs, grids = {}, {}
    t0 = time.perf_counter()
    for p in probs:
        key = (p.n, p.freq)
        if key not in ctxs:
            g = ie.make_grid(p.n, p.h, p.origin)
            ctxs[key] = ie.ie_green_setup(g, ie.ie_medium(p.sigma0, p.freq, 0.0), p.z_bounds)
            grids[key] = g
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    opts = ie.dd_opts(tol=1e-6, adaptive=False, inner_tol_fixed=5e-7, precision=ie.IE_MIXED,
                      max_its=5000, restart=CHOSEN_RESTART)
    data = []
    for p in probs:
        key = (p.n, p.freq)
        E = torch.zeros((3, p.n[2], p.n[1], p.n[0]), dtype=torch.complex128, device="cuda:0")
        data.append((ctxs[key], dict(grid=grids[key], sigma6=torch.from_numpy(p.sigma6).cuda(),
                                     sources=p.sources, E_total=E)))

    def run(sel):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = ie.ie_dd_solve([data[i][0] for i in sel], [data[i][1] for i in sel], opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t, st

    allsel = list(range(len(probs)))
    run(allsel[:12])  # warm-up of every kernel shape
    log("logging run: 128 solves in one call")
    t_all, st = run(allsel)
    mv = sum(s.matvecs32 + s.matvecs64 for s in st)
    worst = max(s.relres[s.sweeps] for s in st)
    nseq = min(args.batch_seq, len(probs))
    t_seq = sum(run([i])[0] for i in range(nseq))
    t_bat, _ = run(list(range(nseq)))
    for c in ctxs.values():
        ie.ie_ctx_destroy(c)
    out = dict(workload="config2: 64 positions x {400 kHz, 2 MHz} = 128 solves, grids "
                        "32^3 / 48x48x64 / 64x64x96 (seed 202), full-domain mixed "
                        f"GMRES({CHOSEN_RESTART}), "
                        "tol 1e-6, one ie_dd_solve call",
               solves=len(probs), groups=len(ctxs), wall_s=round(t_all, 4),
               solves_per_s=round(len(probs) / t_all, 2), matvecs=mv,
               matvecs_per_s=round(mv / t_all, 1), worst_relres=worst,
               green_setup_s=round(t_setup, 3),
               subset=dict(problems=nseq, one_call_each_s=round(t_seq, 4),
                           batched_s=round(t_bat, 4), speedup=round(t_seq / t_bat, 3)))
    log(f"batch: {out}")
    return out


def cpu_baseline(p, gst):
    """The oracle on this host: time restarted GMRES iterations of its full-domain
    contraction-form solve on a bounded sample, then scale to one solve with the iteration and
    restart counts of the GPU run."""
    import scipy.fft
    from oracle import operator, solve as osolve
    from oracle.gmres import gmres
    cores = os.cpu_count() or 1
    with scipy.fft.set_workers(cores):
        t0 = time.perf_counter()
        st = osolve.setup(p)
        t_setup = time.perf_counter() - t0
        b, a, _ = operator.cie_tensors(st.dsig, p.sigma0)
        rhs = np.sqrt(p.sigma0) * st.E0
        x0 = operator.tensor_apply(a, st.E0)
        its = 40
        t0 = time.perf_counter()
        _, info = gmres(lambda v: operator.apply_C(st.Ghat, b, v, p.sigma0, st.n), rhs, x0, 1e-14,
                        CHOSEN_RESTART, its)
        t_sample = time.perf_counter() - t0
        # one iteration = one operator application; each restart adds one more (true residual)
        napp = info["its"] + info["restarts"] + 2
        t_app = t_sample / napp
    est = (gst.its + gst.restarts + 2) * t_app
    return {"value": round(est, 3), "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"oracle FP64 full-domain contraction-form GMRES({CHOSEN_RESTART}) on this "
                      f"host: "
                      f"{info['its']} iterations ({napp} operator applications, "
                      f"{t_sample:.2f} s, {t_app:.3f} s each), scaled to the GPU solve's "
                      f"{gst.its} iterations and {gst.restarts + 1} restarts; oracle setup "
                      f"{t_setup:.2f} s excluded like the GPU setup"}


if __name__ == "__main__":
    main()
