"""Helpers shared by the GPU tests: move synthetic inputs to the device and build contexts
through the C ABI binding.  Nothing here computes any part of the method."""
import sys

import numpy as np


def torch_mod():
    import torch
    return torch


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def context(problem, z_bounds=None, mask=None):
    from paper_2306_17537_amd import ie
    g = ie.make_grid(problem.n, problem.h, problem.origin)
    m = ie.ie_medium(problem.sigma0, problem.freq, 0.0)
    if mask is None:
        mask = ie.IE_FP64 | ie.IE_MIXED
    return ie.ie_green_setup(g, m, z_bounds, mask), g


def field_shape(problem):
    nx, ny, nz = problem.n
    return (3, nz, ny, nx)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
