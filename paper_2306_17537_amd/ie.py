"""Thin ctypes binding of the gfx950 library ``libie_gfx950.so`` (C ABI in ``include/ie.h``).

Functions carry the C names and only marshal arguments: device arrays are passed as raw
pointers (``tensor.data_ptr()``), the stream as ``torch.cuda.current_stream().cuda_stream``.
Every step of the computation runs in the HIP library; there is no host fallback.  A missing
or unloadable library raises ``ImportError`` on first use.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libie_gfx950.so")

IE_OK, IE_ENOCONV, IE_EINVAL, IE_ENOMEM, IE_EDEVICE, IE_ESTATE = 0, 1, -1, -2, -3, -4
IE_FP64, IE_MIXED = 1, 2
IE_CONVENTIONAL, IE_CIE, IE_GREEN_ONLY, IE_SCATTER = 0, 1, 2, 3
IE_GS, IE_JACOBI, IE_FGMRES_GS, IE_FGMRES_JACOBI = 0, 1, 2, 3
IE_INIT_BACKGROUND, IE_INIT_USER, IE_INIT_LEARNED, IE_INIT_ZERO = 0, 1, 2, 3
IE_MAG_DIPOLE, IE_ELEC_DIPOLE = 0, 1
IE_MAX_SWEEPS, IE_MAX_BLOCKS = 128, 16
IE_OPT_GRAPHS, IE_OPT_AUTOTUNE, IE_OPT_FORCE_VARIANT, IE_OPT_GROUP_THREADS = 1, 2, 3, 4


class ie_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("origin", C.c_double * 3)]


class ie_medium(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("freq_hz", C.c_double), ("mu0", C.c_double)]


class ie_source(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("moment", C.c_double * 3), ("kind", C.c_int32)]


class ie_partition(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("z_bounds", C.POINTER(C.c_int32))]


class ie_gmres_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_its", C.c_int32),
                ("precision", C.c_int32), ("form", C.c_int32), ("reorth", C.c_int32)]


class ie_gmres_stats(C.Structure):
    _fields_ = [("its", C.c_int32), ("restarts", C.c_int32), ("refinements", C.c_int32),
                ("matvecs64", C.c_int32), ("matvecs32", C.c_int32), ("graph_cycles", C.c_int32),
                ("relres", C.c_double), ("seconds", C.c_double)]


class ie_dd_opts(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("adaptive", C.c_int32), ("max_sweeps", C.c_int32),
                ("init", C.c_int32), ("tol", C.c_double), ("inner_tol_fixed", C.c_double),
                ("inner", ie_gmres_opts), ("nn", C.c_void_p)]


class ie_dd_stats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("total_its", C.c_int32), ("nblocks", C.c_int32),
                ("block_its", (C.c_int32 * IE_MAX_BLOCKS) * IE_MAX_SWEEPS),
                ("relres", C.c_double * (IE_MAX_SWEEPS + 1)),
                ("matvecs64", C.c_int32), ("matvecs32", C.c_int32),
                ("full_matvecs", C.c_int32), ("learned_used", C.c_int32),
                ("graph_cycles", C.c_int32), ("seconds", C.c_double)]


class ie_problem(C.Structure):
    _fields_ = [("grid", C.POINTER(ie_grid)), ("sigma6", C.c_void_p),
                ("sources", C.POINTER(ie_source)), ("nsources", C.c_int32),
                ("E_total", C.c_void_p), ("E_anom", C.c_void_p)]


class ie_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 96), ("launches", C.c_int32), ("total_ms", C.c_double),
                ("min_ms", C.c_double), ("max_ms", C.c_double), ("bytes_per_launch", C.c_double)]


class ie_nn_config(C.Structure):
    _fields_ = [("in_ch", C.c_int32), ("out_ch", C.c_int32), ("base_ch", C.c_int32),
                ("levels", C.c_int32), ("seed", C.c_uint64)]


_lib = None


def lib():
    """Load the library once; raise ImportError if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2306_17537_amd.build_lib")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.ie_green_setup.argtypes = [C.POINTER(ie_grid), C.POINTER(ie_medium),
                                     C.POINTER(ie_partition), i32, vp, C.POINTER(vp)]
        L.ie_ctx_destroy.argtypes = [vp]
        L.ie_background_field.argtypes = [vp, C.POINTER(ie_source), i32, vp, vp]
        L.ie_matvec.argtypes = [vp, vp, vp, vp, i32, i32, vp]
        L.ie_gmres.argtypes = [vp, vp, vp, vp, C.POINTER(ie_gmres_opts),
                               C.POINTER(ie_gmres_stats), vp]
        L.ie_dd_solve.argtypes = [C.POINTER(vp), i32, C.POINTER(ie_problem),
                                  C.POINTER(ie_dd_opts), C.POINTER(ie_dd_stats), vp]
        L.ie_set_option.argtypes = [i32, i32]
        L.ie_set_option.restype = C.c_int
        L.ie_profile_begin.argtypes = []
        L.ie_profile_end.argtypes = [C.POINTER(ie_kernel_stat), i32, C.POINTER(i32)]
        L.ie_nn_create.argtypes = [C.POINTER(ie_nn_config), vp, C.POINTER(vp)]
        L.ie_nn_destroy.argtypes = [vp]
        L.ie_nn_num_params.argtypes = [vp, C.POINTER(C.c_int64)]
        L.ie_nn_get_params.argtypes = [vp, vp, C.c_int64, i32]
        L.ie_nn_set_params.argtypes = [vp, vp, C.c_int64]
        L.ie_nn_forward.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp]
        L.ie_nn_backward.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp]
        L.ie_nn_train_step.argtypes = [vp, vp, vp, i32, i32, i32, i32, C.c_float,
                                       C.POINTER(C.c_float), vp]
        L.ie_nn_gemm.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp]
        L.ie_nn_guess.argtypes = [vp, vp, vp, vp, vp, C.POINTER(i32), vp]
        L.ie_nn_predict.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ie_ctx_tuning.argtypes = [vp, C.c_char_p, i32]
        L.ie_receivers.argtypes = [vp, vp, C.POINTER(ie_source), i32, vp, vp, i32, vp, vp, vp]
        L.ie_nn_features.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double), vp]
        L.ie_nn_target.argtypes = [vp, vp, vp, vp, vp]
        for f in ("ie_green_setup", "ie_ctx_destroy", "ie_background_field", "ie_matvec",
                  "ie_gmres", "ie_dd_solve", "ie_profile_begin", "ie_profile_end",
                  "ie_nn_create", "ie_nn_destroy", "ie_nn_num_params", "ie_nn_get_params",
                  "ie_nn_set_params", "ie_nn_forward", "ie_nn_backward", "ie_nn_train_step",
                  "ie_nn_gemm", "ie_nn_guess", "ie_nn_features", "ie_nn_target", "ie_nn_predict",
                  "ie_ctx_tuning", "ie_receivers"):
            getattr(L, f).restype = C.c_int
        L.ie_last_error.restype = C.c_char_p
        L.ie_version.restype = C.c_char_p
        _lib = L
    return _lib


class IEError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where} returned {code}: {ie_last_error()}")


def _check(code, where, allow_noconv=False):
    if code < 0 or (code == IE_ENOCONV and not allow_noconv):
        raise IEError(code, where)
    return code


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


def ie_last_error() -> str:
    return lib().ie_last_error().decode()


def ie_version() -> str:
    return lib().ie_version().decode()


def make_grid(n, h, origin) -> ie_grid:
    return ie_grid(int(n[0]), int(n[1]), int(n[2]), float(h), (C.c_double * 3)(*origin))


def make_sources(sources):
    """[(pos, moment, kind)] with kind 'magnetic' / 'electric' (or the IE_ constant)."""
    arr = (ie_source * len(sources))()
    for i, (pos, mom, kind) in enumerate(sources):
        k = kind if isinstance(kind, int) else (IE_MAG_DIPOLE if kind == "magnetic" else IE_ELEC_DIPOLE)
        arr[i] = ie_source((C.c_double * 3)(*pos), (C.c_double * 3)(*mom), k)
    return arr


def ie_green_setup(grid: ie_grid, medium: ie_medium, z_bounds=None, precision_mask=IE_FP64 | IE_MIXED,
                   stream=None):
    """Returns an opaque context handle (int)."""
    part = None
    keep = None
    if z_bounds is not None:
        keep = (C.c_int32 * len(z_bounds))(*z_bounds)
        part = ie_partition(len(z_bounds) - 1, keep)
    out = C.c_void_p()
    rc = lib().ie_green_setup(C.byref(grid), C.byref(medium),
                              C.byref(part) if part is not None else None,
                              precision_mask, _stream(stream), C.byref(out))
    _check(rc, "ie_green_setup")
    return out.value


def ie_ctx_destroy(ctx):
    return _check(lib().ie_ctx_destroy(C.c_void_p(ctx)), "ie_ctx_destroy")


def ie_background_field(ctx, sources, E0, stream=None):
    src = make_sources(sources) if not isinstance(sources, C.Array) else sources
    return _check(lib().ie_background_field(C.c_void_p(ctx), src, len(src), _ptr(E0),
                                            _stream(stream)), "ie_background_field")


def ie_matvec(ctx, sigma6, x, y, form=IE_CONVENTIONAL, precision=IE_FP64, stream=None):
    return _check(lib().ie_matvec(C.c_void_p(ctx), _ptr(sigma6), _ptr(x), _ptr(y), form,
                                  precision, _stream(stream)), "ie_matvec")


def ie_gmres(ctx, sigma6, b, x, tol=1e-6, restart=10, max_its=2000, precision=IE_FP64,
             form=IE_CIE, stream=None, allow_noconv=False, reorth=0):
    """Solve in place (x holds the initial guess).  Returns (status, ie_gmres_stats)."""
    opts = ie_gmres_opts(tol, restart, max_its, precision, form, reorth)
    st = ie_gmres_stats()
    rc = lib().ie_gmres(C.c_void_p(ctx), _ptr(sigma6), _ptr(b), _ptr(x), C.byref(opts),
                        C.byref(st), _stream(stream))
    _check(rc, "ie_gmres", allow_noconv)
    return rc, st


def dd_opts(scheme=IE_GS, adaptive=True, tol=1e-6, inner_tol_fixed=1e-6, max_sweeps=50,
            init=IE_INIT_BACKGROUND, restart=10, max_its=5000, precision=IE_FP64, form=IE_CIE,
            nn=None, reorth=0) -> ie_dd_opts:
    return ie_dd_opts(scheme, 1 if adaptive else 0, max_sweeps, init, tol, inner_tol_fixed,
                      ie_gmres_opts(0.0, restart, max_its, precision, form, reorth),
                      C.c_void_p(nn) if nn else None)


def ie_dd_solve(ctxs, problems, opts: ie_dd_opts, stream=None, allow_noconv=False):
    """problems: list of dicts with keys grid (ie_grid), sigma6, sources, E_total, E_anom.
    Returns (status, [ie_dd_stats])."""
    n = len(problems)
    carr = (C.c_void_p * n)(*ctxs)
    parr = (ie_problem * n)()
    keep = []
    for i, p in enumerate(problems):
        src = make_sources(p["sources"])
        g = p["grid"]
        keep += [src, g]
        parr[i] = ie_problem(C.pointer(g), _ptr(p["sigma6"]), src, len(src),
                             _ptr(p["E_total"]), _ptr(p.get("E_anom")))
    stats = (ie_dd_stats * n)()
    rc = lib().ie_dd_solve(carr, n, parr, C.byref(opts), stats, _stream(stream))
    _check(rc, "ie_dd_solve", allow_noconv)
    return rc, list(stats)


def ie_profile_begin():
    return _check(lib().ie_profile_begin(), "ie_profile_begin")


def ie_profile_end(cap=256):
    """Returns a list of dicts (name, launches, total_ms, min_ms, max_ms, bytes_per_launch)."""
    arr = (ie_kernel_stat * cap)()
    n = C.c_int32(0)
    _check(lib().ie_profile_end(arr, cap, C.byref(n)), "ie_profile_end")
    out = []
    for k in arr[:min(cap, n.value)]:
        out.append(dict(name=k.name.decode(), launches=k.launches, total_ms=k.total_ms,
                        min_ms=k.min_ms, max_ms=k.max_ms, bytes_per_launch=k.bytes_per_launch))
    return out


def ie_receivers(ctx, sigma6, sources, E, rx, stream=None):
    """Magnetic field at receivers rx [(x, y, z), ...]; returns (H, Ha) as numpy [nrx, 3]."""
    import numpy as np
    src = make_sources(sources) if not isinstance(sources, C.Array) else sources
    pts = np.ascontiguousarray(rx, dtype=np.float64).reshape(-1, 3)
    H = np.empty((len(pts), 3), dtype=np.complex128)
    Ha = np.empty_like(H)
    _check(lib().ie_receivers(C.c_void_p(ctx), _ptr(sigma6), src, len(src), _ptr(E),
                              pts.ctypes.data, len(pts), H.ctypes.data, Ha.ctypes.data,
                              _stream(stream)), "ie_receivers")
    return H, Ha


def ie_ctx_tuning(ctx):
    """The autotuner's per-pass decisions for a context (list of dicts)."""
    import json
    buf = C.create_string_buffer(1 << 16)
    _check(lib().ie_ctx_tuning(C.c_void_p(ctx), buf, len(buf)), "ie_ctx_tuning")
    return json.loads(buf.value.decode())


def ie_set_option(option, value):
    return _check(lib().ie_set_option(option, value), "ie_set_option")


# ----------------------------------------------------------------------------------------
# learned initial guess (network); x / dy / target / y are device tensors: x bfloat16
# channels-last [batch, nz, ny, nx, in_ch], the others float32 [batch, nz, ny, nx, out_ch]
# ----------------------------------------------------------------------------------------
def ie_nn_create(in_ch=14, out_ch=6, base_ch=32, levels=4, seed=0, stream=None):
    cfg = ie_nn_config(in_ch, out_ch, base_ch, levels, seed)
    out = C.c_void_p()
    _check(lib().ie_nn_create(C.byref(cfg), _stream(stream), C.byref(out)), "ie_nn_create")
    return out.value


def ie_nn_destroy(nn):
    return _check(lib().ie_nn_destroy(C.c_void_p(nn)), "ie_nn_destroy")


def ie_nn_num_params(nn):
    n = C.c_int64()
    _check(lib().ie_nn_num_params(C.c_void_p(nn), C.byref(n)), "ie_nn_num_params")
    return n.value


def ie_nn_get_params(nn, which=0):
    """float32 numpy copy: which = 0 weights, 1 gradients of the last backward."""
    import numpy as np
    a = np.empty(ie_nn_num_params(nn), dtype=np.float32)
    _check(lib().ie_nn_get_params(C.c_void_p(nn), a.ctypes.data, a.size, which), "ie_nn_get_params")
    return a


def ie_nn_set_params(nn, params):
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().ie_nn_set_params(C.c_void_p(nn), a.ctypes.data, a.size), "ie_nn_set_params")


def ie_nn_forward(nn, x, y, stream=None):
    b, nz, ny, nx = x.shape[:4]
    return _check(lib().ie_nn_forward(C.c_void_p(nn), _ptr(x), b, nz, ny, nx, _ptr(y),
                                      _stream(stream)), "ie_nn_forward")


def ie_nn_backward(nn, x, dy, y, stream=None):
    b, nz, ny, nx = x.shape[:4]
    return _check(lib().ie_nn_backward(C.c_void_p(nn), _ptr(x), _ptr(dy), b, nz, ny, nx, _ptr(y),
                                       _stream(stream)), "ie_nn_backward")


def ie_nn_train_step(nn, x, target, lr, stream=None):
    """One Adam step on the mean squared error; returns the loss before the step."""
    b, nz, ny, nx = x.shape[:4]
    loss = C.c_float()
    _check(lib().ie_nn_train_step(C.c_void_p(nn), _ptr(x), _ptr(target), b, nz, ny, nx,
                                  C.c_float(lr), C.byref(loss), _stream(stream)),
           "ie_nn_train_step")
    return loss.value


def ie_nn_gemm(A, B, Cout, M, N, K, a_trans=0, b_trans=0, splits=1, stream=None):
    return _check(lib().ie_nn_gemm(_ptr(A), _ptr(B), _ptr(Cout), M, N, K, a_trans, b_trans, splits,
                                   _stream(stream)), "ie_nn_gemm")


def ie_nn_features(ctx, sigma6, b, x, stream=None):
    """Features into x (bfloat16 [nz, ny, nx, 14]); returns rms(b)."""
    r = C.c_double(0)
    _check(lib().ie_nn_features(C.c_void_p(ctx), _ptr(sigma6), _ptr(b), _ptr(x), C.byref(r),
                                _stream(stream)), "ie_nn_features")
    return r.value


def ie_nn_target(ctx, b, E, y, stream=None):
    return _check(lib().ie_nn_target(C.c_void_p(ctx), _ptr(b), _ptr(E), _ptr(y), _stream(stream)),
                  "ie_nn_target")


def ie_nn_predict(ctx, nn, sigma6, b, x, stream=None):
    """The network's (unjudged) guess for the full grid into x."""
    return _check(lib().ie_nn_predict(C.c_void_p(ctx), C.c_void_p(nn), _ptr(sigma6), _ptr(b),
                                      _ptr(x), _stream(stream)), "ie_nn_predict")


def ie_nn_guess(ctx, nn, sigma6, b, x, stream=None):
    """Learned guess on the full grid; returns 1 (learned), 0 (default kept) or 2 (zero)."""
    acc = C.c_int32(0)
    _check(lib().ie_nn_guess(C.c_void_p(ctx), C.c_void_p(nn), _ptr(sigma6), _ptr(b), _ptr(x),
                             C.byref(acc), _stream(stream)), "ie_nn_guess")
    return acc.value
