"""Learned initial guess for the inner solves: training data made by this solver, training with
the library's own network kernels (``ie_nn_train_step``), evaluation, and weight files.

The network maps solver features (contraction-form contrast tensor, right-hand side scaled by
its rms with its global phase removed, k0 h) to the scaled anomalous field (E - b) / rms(b) of
the block system (I - G dsigma) E = b, rotated by the same phase.  Training samples are single-block 32^3 problems whose right-hand side is
the background field of a dipole outside the block, so that b plays the part of the coupled
right-hand side a sub-domain sees.  Every solve, feature and gradient here runs in the HIP
library; PyTorch only holds device memory and gathers mini-batches.

Command line (writes the weight file and a JSON log):
    python -m paper_2306_17537_amd.guess train --samples 2000 --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import ie

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(_HERE, "weights", "guess_c32_l4.npy")
NET = dict(in_ch=14, out_ch=6, base_ch=32, levels=4)


def _say(msg):
    print(f"[guess] {msg}", flush=True)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the learned guess runs on the GPU only")
    return torch


# ----------------------------------------------------------------------------------------
# weights
# ----------------------------------------------------------------------------------------
def save_weights(nn, path):
    """Store the float32 master weights rounded to bfloat16 (the values inference uses)."""
    w = ie.ie_nn_get_params(nn)
    u = w.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.save(path, u, allow_pickle=False)


def load_weights(nn, path=WEIGHTS):
    u = np.load(path, allow_pickle=False)
    if u.dtype != np.uint16 or u.size != ie.ie_nn_num_params(nn):
        raise ValueError(f"{path}: expected {ie.ie_nn_num_params(nn)} bfloat16 weights")
    ie.ie_nn_set_params(nn, (u.astype(np.uint32) << 16).view(np.float32))


def create(path=WEIGHTS, seed=0):
    """The guess network, with trained weights from `path` when given (None: fresh weights)."""
    nn = ie.ie_nn_create(NET["in_ch"], NET["out_ch"], NET["base_ch"], NET["levels"], seed)
    if path is not None:
        load_weights(nn, path)
    return nn


# ----------------------------------------------------------------------------------------
# training data
# ----------------------------------------------------------------------------------------
def generate(problems, tol=1e-6, batch=64, precision=ie.IE_MIXED, max_its=3000, keep_below=1e-4):
    """Solve every single-block problem with the library and return device tensors
    (X bfloat16 [S', nz, ny, nx, 14], T float32 [S', nz, ny, nx, 6]) of the S' problems whose
    solve reached relative residual `keep_below` within the iteration cap, plus statistics."""
    torch = _torch()
    S = len(problems)
    nx, ny, nz = problems[0].n
    X = torch.empty((S, nz, ny, nx, 14), dtype=torch.bfloat16, device="cuda:0")
    T = torch.empty((S, nz, ny, nx, 6), dtype=torch.float32, device="cuda:0")
    ctxs = {}
    its = []
    ok = np.zeros(S, dtype=bool)
    relres = np.zeros(S)
    t0 = time.time()
    order = sorted(range(S), key=lambda i: problems[i].freq)
    for c0 in range(0, S, batch):
        chunk = [i for i in order[c0:c0 + batch]]
        by_f = {}
        for i in chunk:
            by_f.setdefault(problems[i].freq, []).append(i)
        for f, ids in by_f.items():
            p0 = problems[ids[0]]
            if f not in ctxs:
                g = ie.make_grid(p0.n, p0.h, p0.origin)
                ctxs[f] = (ie.ie_green_setup(g, ie.ie_medium(p0.sigma0, f, 0.0), (0, nz),
                                             ie.IE_FP64 | ie.IE_MIXED), g)
            ctx, g = ctxs[f]
            sig = [torch.from_numpy(problems[i].sigma6).to("cuda:0") for i in ids]
            E = [torch.empty((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0") for _ in ids]
            probs = [dict(grid=g, sigma6=sig[k], sources=problems[i].sources, E_total=E[k])
                     for k, i in enumerate(ids)]
            opts = ie.dd_opts(scheme=ie.IE_GS, adaptive=False, tol=tol, inner_tol_fixed=0.5 * tol,
                              max_sweeps=2, precision=precision, form=ie.IE_CIE, max_its=max_its)
            _, st = ie.ie_dd_solve([ctx] * len(ids), probs, opts, allow_noconv=True)
            E0 = torch.empty((3, nz, ny, nx), dtype=torch.complex128, device="cuda:0")
            for k, i in enumerate(ids):
                its.append(st[k].total_its)
                relres[i] = st[k].relres[st[k].sweeps]
                ok[i] = relres[i] <= keep_below
                ie.ie_background_field(ctx, problems[i].sources, E0)
                ie.ie_nn_features(ctx, sig[k], E0, X[i])
                ie.ie_nn_target(ctx, E0, E[k], T[i])
        _say(f"generated {min(c0 + batch, S)}/{S} solves in {time.time() - t0:.1f} s")
    for ctx, _ in ctxs.values():
        ie.ie_ctx_destroy(ctx)
    keep = torch.from_numpy(np.nonzero(ok)[0]).to("cuda:0")
    q = np.percentile(its, [50, 90, 100])
    stats = dict(seconds=time.time() - t0, solves=S, kept=int(ok.sum()),
                 its_p50=float(q[0]), its_p90=float(q[1]), its_max=float(q[2]),
                 worst_relres=float(relres.max()))
    bad = [(problems[i].name, problems[i].freq, float(relres[i])) for i in np.nonzero(~ok)[0][:8]]
    if bad:
        stats["dropped_examples"] = bad
    return X[keep].contiguous(), T[keep].contiguous(), stats


# ----------------------------------------------------------------------------------------
# training
# ----------------------------------------------------------------------------------------
def evaluate_loss(nn, X, T, batch=8):
    torch = _torch()
    y = torch.empty_like(T[:batch])
    tot, cnt = 0.0, 0
    for i in range(0, X.shape[0], batch):
        xb, tb = X[i:i + batch], T[i:i + batch]
        yb = y[:xb.shape[0]]
        ie.ie_nn_forward(nn, xb, yb)
        tot += float(((yb - tb) ** 2).sum())
        cnt += tb.numel()
    return tot / cnt


def train(nn, X, T, Xv=None, Tv=None, epochs=12, batch=8, lr=1e-3, lr_min=2e-5, seed=0):
    """Adam on the mean squared error with a cosine learning-rate decay; returns the log."""
    torch = _torch()
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    S = X.shape[0]
    steps = epochs * (S // batch)
    log = dict(train=[], val=[], seconds=0.0, steps=steps)
    t0 = time.time()
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(S, device="cuda:0", generator=gen)
        run = 0.0
        for i in range(0, S - batch + 1, batch):
            idx = perm[i:i + batch]
            a = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * k / steps))
            run += ie.ie_nn_train_step(nn, X[idx].contiguous(), T[idx].contiguous(), a)
            k += 1
        log["train"].append(run / (S // batch))
        if Xv is not None:
            log["val"].append(evaluate_loss(nn, Xv, Tv))
        _say(f"epoch {ep + 1}/{epochs}: train {log['train'][-1]:.4e}"
             + (f", val {log['val'][-1]:.4e}" if Xv is not None else "")
             + f"  ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    log["seconds"] = time.time() - t0
    return log


# ----------------------------------------------------------------------------------------
# the learned start with zero-start GMRES as judge
# ----------------------------------------------------------------------------------------
def solve_learned_start(ctx, nn, sigma6, b, x, tol=1e-6, restart=10, precision=ie.IE_MIXED):
    """One restart cycle of GMRES from the network's guess and one from zero; x receives the
    state of whichever cycle reached the smaller residual (the caller continues from it).
    Returns 1 if the learned start won."""
    torch = _torch()
    xl = torch.empty_like(x)
    ie.ie_nn_predict(ctx, nn, sigma6, b, xl)
    x.zero_()
    _, sl = ie.ie_gmres(ctx, sigma6, b, xl, tol=tol, restart=restart, max_its=restart,
                        precision=precision, form=ie.IE_CIE, allow_noconv=True)
    _, sz = ie.ie_gmres(ctx, sigma6, b, x, tol=tol, restart=restart, max_its=restart,
                        precision=precision, form=ie.IE_CIE, allow_noconv=True)
    if sl.relres < sz.relres:
        x.copy_(xl)
        return 1
    return 0


# ----------------------------------------------------------------------------------------
# evaluation: what the learned start gains over zero and background starts
# ----------------------------------------------------------------------------------------
def evaluate(nn, problems, tol=1e-6, precision=ie.IE_MIXED, restart=10):
    """For problems that share grid, frequency and partition: block Gauss-Seidel with a fixed
    inner tolerance `tol` (every block solved to `tol`) and full-domain GMRES, each from a zero
    start, the background field and the learned guess.  Returns per-variant statistics."""
    torch = _torch()
    p0 = problems[0]
    nx, ny, nz = p0.n
    g = ie.make_grid(p0.n, p0.h, p0.origin)
    ctx = ie.ie_green_setup(g, ie.ie_medium(p0.sigma0, p0.freq, 0.0), p0.z_bounds,
                            ie.IE_FP64 | ie.IE_MIXED)
    out = {}
    try:
        sig = [torch.from_numpy(p.sigma6).to("cuda:0") for p in problems]
        shape = (3, nz, ny, nx)
        M = len(p0.z_bounds) - 1
        # domain decomposition
        for name, init in (("zero", ie.IE_INIT_ZERO), ("background", ie.IE_INIT_BACKGROUND),
                           ("learned", ie.IE_INIT_LEARNED)):
            E = [torch.zeros(shape, dtype=torch.complex128, device="cuda:0") for _ in problems]
            probs = [dict(grid=g, sigma6=sig[k], sources=p.sources, E_total=E[k])
                     for k, p in enumerate(problems)]
            opts = ie.dd_opts(scheme=ie.IE_GS, adaptive=False, tol=tol, inner_tol_fixed=tol,
                              max_sweeps=60, init=init, precision=precision, form=ie.IE_CIE,
                              restart=restart, nn=nn if init == ie.IE_INIT_LEARNED else None)
            torch.cuda.synchronize()
            t0 = time.time()
            _, st = ie.ie_dd_solve([ctx] * len(problems), probs, opts, allow_noconv=True)
            torch.cuda.synchronize()
            secs = time.time() - t0
            out[f"dd_gs_{name}"] = dict(
                seconds=secs,
                first_sweep_its=[int(sum(s.block_its[0][i] for i in range(M))) for s in st],
                total_its=[int(s.total_its) for s in st], sweeps=[int(s.sweeps) for s in st],
                learned_used=[int(s.learned_used) for s in st],
                relres=[float(s.relres[s.sweeps]) for s in st])
            _say(f"dd {name}: {secs:.2f} s, first-sweep its "
                 f"{np.mean(out[f'dd_gs_{name}']['first_sweep_its']):.1f}, total its "
                 f"{np.mean(out[f'dd_gs_{name}']['total_its']):.1f}")
        # full-domain GMRES: zero start, background start, and the learned start judged against
        # the zero start after one restart cycle each (the better one continues)
        for name in ("zero", "background", "learned"):
            its, secs, rel, acc = [], [], [], []
            for k, p in enumerate(problems):
                E0 = torch.empty(shape, dtype=torch.complex128, device="cuda:0")
                x = torch.zeros(shape, dtype=torch.complex128, device="cuda:0")
                torch.cuda.synchronize()
                t0 = time.time()
                ie.ie_background_field(ctx, p.sources, E0)
                used = 0
                if name == "background":
                    x.copy_(E0)
                elif name == "learned":
                    used = solve_learned_start(ctx, nn, sig[k], E0, x, tol, restart, precision)
                    acc.append(used)
                _, st = ie.ie_gmres(ctx, sig[k], E0, x, tol=tol, restart=restart,
                                    precision=precision, form=ie.IE_CIE, max_its=5000,
                                    allow_noconv=True)
                torch.cuda.synchronize()
                secs.append(time.time() - t0)
                its.append(int(st.its) + (2 * restart if name == "learned" else 0))
                rel.append(float(st.relres))
            out[f"full_{name}"] = dict(seconds=secs, its=its, relres=rel, learned_used=acc)
            _say(f"full {name}: mean {np.mean(secs) * 1e3:.1f} ms, its {np.mean(its):.1f}")
    finally:
        ie.ie_ctx_destroy(ctx)
    return out


def main(argv=None):
    import synth
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--samples", type=int, default=2000)
    tr.add_argument("--val", type=int, default=64)
    tr.add_argument("--epochs", type=int, default=12)
    tr.add_argument("--batch", type=int, default=8)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--out", default=WEIGHTS)
    tr.add_argument("--log", default=None)
    tr.add_argument("--eval", type=int, default=0, help="evaluation models after training")
    ev = sub.add_parser("eval")
    ev.add_argument("--weights", default=WEIGHTS)
    ev.add_argument("--models", type=int, default=16)
    ev.add_argument("--log", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "eval":
        _torch()
        nn = create(a.weights)
        try:
            res = evaluate(nn, list(synth.config4_eval(count=a.models)))
        finally:
            ie.ie_nn_destroy(nn)
        if a.log:
            with open(a.log, "w") as f:
                json.dump(res, f, indent=1)
        return 0
    _torch()
    _say(f"building {a.samples} training and {a.val} validation models")
    train_p = list(synth.config4_train(count=a.samples))
    val_p = list(synth.config4_train(start=45000, count=a.val))
    X, T, gs = generate(train_p)
    _say(f"training data: {gs}")
    Xv, Tv, vs = generate(val_p)
    zero_val = float((Tv.double() ** 2).mean())
    _say(f"validation loss of the zero prediction: {zero_val:.4e}")
    nn = create(path=None, seed=1)
    try:
        log = train(nn, X, T, Xv, Tv, epochs=a.epochs, batch=a.batch, lr=a.lr)
        del X, T
        save_weights(nn, a.out)
        log.update(generation=gs, net=NET, samples=a.samples, batch=a.batch, lr=a.lr,
                   val_zero=zero_val)
        _say(f"weights -> {a.out}")
        if a.eval:
            load_weights(nn, a.out)  # evaluate exactly the stored (bfloat16) weights
            log["eval"] = evaluate(nn, list(synth.config4_eval(count=a.eval)))
        if a.log:
            with open(a.log, "w") as f:
                json.dump(log, f, indent=1)
    finally:
        ie.ie_nn_destroy(nn)
    return 0


if __name__ == "__main__":
    sys.exit(main())
