"""Thin ctypes binding of the gfx950 library ``libie_gfx950.so`` (C ABI in ``include/ie.h``).

Functions carry the C names and only marshal arguments: device arrays are passed as raw
pointers (``tensor.data_ptr()``), the stream as ``torch.cuda.current_stream().cuda_stream``.
Before any call each array is checked against what the header states (a contiguous GPU tensor
of the stated dtype, element count and, for arrays of a context, the context's device), since
the library cannot check sizes behind a pointer; a mismatch raises ValueError.
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
IE_OPT_FFT_LENGTHS = 5
IE_RESID_ALL, IE_RESID_ANOMALOUS = 0, 1


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
                ("inner", ie_gmres_opts), ("nn", C.c_void_p), ("residual_cells", C.c_int32)]


class ie_dd_stats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("total_its", C.c_int32), ("nblocks", C.c_int32),
                ("block_its", (C.c_int32 * IE_MAX_BLOCKS) * IE_MAX_SWEEPS),
                ("relres", C.c_double * (IE_MAX_SWEEPS + 1)),
                ("matvecs64", C.c_int32), ("matvecs32", C.c_int32),
                ("full_matvecs", C.c_int32), ("learned_used", C.c_int32),
                ("graph_cycles", C.c_int32), ("seconds", C.c_double),
                ("best_sweep", C.c_int32), ("diverged", C.c_int32)]


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
        L.ie_matvec_noalloc.argtypes = [vp, vp, vp, vp, i32, i32, vp]
        L.ie_gmres.argtypes = [vp, vp, vp, vp, C.POINTER(ie_gmres_opts),
                               C.POINTER(ie_gmres_stats), vp]
        L.ie_dd_solve.argtypes = [C.POINTER(vp), i32, C.POINTER(ie_problem),
                                  C.POINTER(ie_dd_opts), C.POINTER(ie_dd_stats), vp]
        L.ie_set_option.argtypes = [i32, i32]
        L.ie_set_option.restype = C.c_int
        for f in (L.ie_tuning_save, L.ie_tuning_load):
            f.argtypes = [C.c_char_p]
            f.restype = C.c_int
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
                  "ie_matvec_noalloc",
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


# what the binding knows of each live handle, for the argument checks below:
# context -> ((nx, ny, nz), device index); network -> (in_ch, out_ch)
_CTX = {}
_NN = {}


def _dtype(name):
    import torch
    return getattr(torch, name)


def _arg(t, what, dtypes, numel=None, optional=False):
    """Check that `t` is a contiguous tensor of one of `dtypes` (torch dtype names) with `numel`
    elements; returns (what, t), or None for an omitted optional array.  Raises ValueError (the
    library cannot check sizes behind a raw pointer)."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{what}: a device tensor is required")
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    allowed = [_dtype(d) for d in dtypes]
    if t.dtype not in allowed:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {' or '.join(map(str, allowed))}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, expected {numel}")
    return what, t


def _ptrs(device, *args):
    """Pointers of checked arrays (from _arg) after checking that each is a GPU tensor on
    `device` (any device if None, then all on the first one's)."""
    out = []
    for a in args:
        if a is None:
            out.append(None)
            continue
        what, t = a
        if t.device.type != "cuda":
            raise ValueError(f"{what}: must be a GPU tensor, not on {t.device}")
        if device is None:
            device = t.device.index
        if t.device.index != device:
            raise ValueError(f"{what}: on cuda:{t.device.index}, expected cuda:{device}")
        out.append(C.c_void_p(t.data_ptr()))
    return out


def _ctx_cells(ctx):
    """(cell count, device) of a context made by this binding, else (None, None)."""
    info = _CTX.get(ctx)
    if info is None:
        return None, None
    (nx, ny, nz), device = info
    return nx * ny * nz, device


def _field(ctx, t, what, prec=IE_FP64, optional=False):
    N = _ctx_cells(ctx)[0]
    dt = ("complex128",) if prec == IE_FP64 else ("complex64",)
    return _arg(t, what, dt, None if N is None else 3 * N, optional)


def _tensor6(ctx, t, what="sigma6", optional=False):
    N = _ctx_cells(ctx)[0]
    return _arg(t, what, ("float64",), None if N is None else 6 * N, optional)


def _dev_of(ctx):
    return _ctx_cells(ctx)[1]


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
    import torch
    _CTX[out.value] = ((grid.nx, grid.ny, grid.nz), torch.cuda.current_device())
    return out.value


def ie_ctx_destroy(ctx):
    _CTX.pop(ctx, None)
    return _check(lib().ie_ctx_destroy(C.c_void_p(ctx)), "ie_ctx_destroy")


def ie_background_field(ctx, sources, E0, stream=None):
    src = make_sources(sources) if not isinstance(sources, C.Array) else sources
    (e0,) = _ptrs(_dev_of(ctx), _field(ctx, E0, "E0"))
    return _check(lib().ie_background_field(C.c_void_p(ctx), src, len(src), e0,
                                            _stream(stream)), "ie_background_field")


def _matvec_args(ctx, sigma6, x, y, form, precision):
    return _ptrs(_dev_of(ctx), _tensor6(ctx, sigma6, optional=form == IE_GREEN_ONLY),
                 _field(ctx, x, "x", precision), _field(ctx, y, "y", precision))


def ie_matvec(ctx, sigma6, x, y, form=IE_CONVENTIONAL, precision=IE_FP64, stream=None):
    s6, xp, yp = _matvec_args(ctx, sigma6, x, y, form, precision)
    return _check(lib().ie_matvec(C.c_void_p(ctx), s6, xp, yp, form, precision, _stream(stream)),
                  "ie_matvec")


def ie_matvec_noalloc(ctx, sigma6, x, y, form=IE_CONVENTIONAL, precision=IE_FP64, stream=None):
    s6, xp, yp = _matvec_args(ctx, sigma6, x, y, form, precision)
    return _check(lib().ie_matvec_noalloc(C.c_void_p(ctx), s6, xp, yp, form, precision,
                                          _stream(stream)), "ie_matvec_noalloc")


def ie_gmres(ctx, sigma6, b, x, tol=1e-6, restart=10, max_its=2000, precision=IE_FP64,
             form=IE_CIE, stream=None, allow_noconv=False, reorth=0):
    """Solve in place (x holds the initial guess).  Returns (status, ie_gmres_stats)."""
    opts = ie_gmres_opts(tol, restart, max_its, precision, form, reorth)
    st = ie_gmres_stats()
    s6, bp, xp = _ptrs(_dev_of(ctx), _tensor6(ctx, sigma6), _field(ctx, b, "b"),
                       _field(ctx, x, "x"))
    rc = lib().ie_gmres(C.c_void_p(ctx), s6, bp, xp, C.byref(opts), C.byref(st),
                        _stream(stream))
    _check(rc, "ie_gmres", allow_noconv)
    return rc, st


def dd_opts(scheme=IE_GS, adaptive=True, tol=1e-6, inner_tol_fixed=1e-6, max_sweeps=50,
            init=IE_INIT_BACKGROUND, restart=10, max_its=5000, precision=IE_FP64, form=IE_CIE,
            nn=None, reorth=0, residual_cells=0) -> ie_dd_opts:
    return ie_dd_opts(scheme, 1 if adaptive else 0, max_sweeps, init, tol, inner_tol_fixed,
                      ie_gmres_opts(0.0, restart, max_its, precision, form, reorth),
                      C.c_void_p(nn) if nn else None, residual_cells)


def ie_dd_solve(ctxs, problems, opts: ie_dd_opts, stream=None, allow_noconv=False):
    """problems: list of dicts with keys grid (ie_grid), sigma6, sources, E_total, E_anom.
    Returns (status, [ie_dd_stats])."""
    n = len(problems)
    carr = (C.c_void_p * n)(*ctxs)
    parr = (ie_problem * n)()
    keep = []
    checked = []
    for i, p in enumerate(problems):
        src = make_sources(p["sources"])
        g = p["grid"]
        keep += [src, g]
        N = g.nx * g.ny * g.nz
        checked.append((i, _arg(p["sigma6"], f"problem {i} sigma6", ("float64",), 6 * N),
                        _arg(p["E_total"], f"problem {i} E_total", ("complex128",), 3 * N),
                        _arg(p.get("E_anom"), f"problem {i} E_anom", ("complex128",), 3 * N,
                             optional=True), src, g))
    for i, s6, et, ea, src, g in checked:
        s6p, etp, eap = _ptrs(_dev_of(ctxs[i]), s6, et, ea)
        parr[i] = ie_problem(C.pointer(g), s6p, src, len(src), etp, eap)
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
    s6, ep = _ptrs(_dev_of(ctx), _tensor6(ctx, sigma6), _field(ctx, E, "E"))
    _check(lib().ie_receivers(C.c_void_p(ctx), s6, src, len(src), ep,
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


def ie_tuning_save(path):
    """Write the autotuner's cache to a JSON file."""
    return _check(lib().ie_tuning_save(os.fsencode(path)), "ie_tuning_save")


def ie_tuning_load(path):
    """Add the entries of a file written by ie_tuning_save to the autotuner's cache."""
    return _check(lib().ie_tuning_load(os.fsencode(path)), "ie_tuning_load")


# ----------------------------------------------------------------------------------------
# learned initial guess (network); x / dy / target / y are device tensors: x bfloat16
# channels-last [batch, nz, ny, nx, in_ch], the others float32 [batch, nz, ny, nx, out_ch]
# ----------------------------------------------------------------------------------------
def ie_nn_create(in_ch=14, out_ch=6, base_ch=32, levels=4, seed=0, stream=None):
    cfg = ie_nn_config(in_ch, out_ch, base_ch, levels, seed)
    out = C.c_void_p()
    _check(lib().ie_nn_create(C.byref(cfg), _stream(stream), C.byref(out)), "ie_nn_create")
    _NN[out.value] = (in_ch, out_ch)
    return out.value


def ie_nn_destroy(nn):
    _NN.pop(nn, None)
    return _check(lib().ie_nn_destroy(C.c_void_p(nn)), "ie_nn_destroy")


def _nn_io(nn, x, y, ywhat="y", ydtype="float32"):
    """Pointers of a network input x (bfloat16 [batch, nz, ny, nx, in_ch]) and an output-shaped
    tensor y ([batch, nz, ny, nx, out_ch]), checked; returns (b, nz, ny, nx, xp, yp)."""
    if x is None or x.dim() != 5:
        raise ValueError("x: expected a [batch, nz, ny, nx, channels] tensor")
    b, nz, ny, nx = (int(v) for v in x.shape[:4])
    cin, cout = _NN.get(nn, (None, None))
    cells = b * nz * ny * nx
    xa = _arg(x, "x", ("bfloat16",), None if cin is None else cells * cin)
    ya = _arg(y, ywhat, (ydtype,), None if cout is None else cells * cout)
    return b, nz, ny, nx, xa, ya


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
    b, nz, ny, nx, xa, ya = _nn_io(nn, x, y)
    xp, yp = _ptrs(None, xa, ya)
    return _check(lib().ie_nn_forward(C.c_void_p(nn), xp, b, nz, ny, nx, yp, _stream(stream)),
                  "ie_nn_forward")


def ie_nn_backward(nn, x, dy, y, stream=None):
    b, nz, ny, nx, xa, ya = _nn_io(nn, x, y)
    dya = _nn_io(nn, x, dy, "dy")[5]
    xp, yp, dyp = _ptrs(None, xa, ya, dya)
    return _check(lib().ie_nn_backward(C.c_void_p(nn), xp, dyp, b, nz, ny, nx, yp,
                                       _stream(stream)), "ie_nn_backward")


def ie_nn_train_step(nn, x, target, lr, stream=None):
    """One Adam step on the mean squared error; returns the loss before the step."""
    b, nz, ny, nx, xa, ta = _nn_io(nn, x, target, "target")
    xp, tp = _ptrs(None, xa, ta)
    loss = C.c_float()
    _check(lib().ie_nn_train_step(C.c_void_p(nn), xp, tp, b, nz, ny, nx, C.c_float(lr),
                                  C.byref(loss), _stream(stream)), "ie_nn_train_step")
    return loss.value


def ie_nn_gemm(A, B, Cout, M, N, K, a_trans=0, b_trans=0, splits=1, stream=None):
    ap, bp, cp = _ptrs(None, _arg(A, "A", ("bfloat16", "int16"), M * K),
                       _arg(B, "B", ("bfloat16", "int16"), K * N),
                       _arg(Cout, "C", ("float32",), M * N))
    return _check(lib().ie_nn_gemm(ap, bp, cp, M, N, K, a_trans, b_trans, splits,
                                   _stream(stream)), "ie_nn_gemm")


def ie_nn_features(ctx, sigma6, b, x, stream=None):
    """Features into x (bfloat16 [nz, ny, nx, 14]); returns rms(b)."""
    N, d = _ctx_cells(ctx)
    s6, bp, xp = _ptrs(d, _tensor6(ctx, sigma6), _field(ctx, b, "b"),
                       _arg(x, "x", ("bfloat16",), None if N is None else 14 * N))
    r = C.c_double(0)
    _check(lib().ie_nn_features(C.c_void_p(ctx), s6, bp, xp, C.byref(r), _stream(stream)),
           "ie_nn_features")
    return r.value


def ie_nn_target(ctx, b, E, y, stream=None):
    N, d = _ctx_cells(ctx)
    bp, ep, yp = _ptrs(d, _field(ctx, b, "b"), _field(ctx, E, "E"),
                       _arg(y, "y", ("float32",), None if N is None else 6 * N))
    return _check(lib().ie_nn_target(C.c_void_p(ctx), bp, ep, yp, _stream(stream)),
                  "ie_nn_target")


def ie_nn_predict(ctx, nn, sigma6, b, x, stream=None):
    """The network's (unjudged) guess for the full grid into x."""
    s6, bp, xp = _ptrs(_dev_of(ctx), _tensor6(ctx, sigma6), _field(ctx, b, "b"),
                       _field(ctx, x, "x"))
    return _check(lib().ie_nn_predict(C.c_void_p(ctx), C.c_void_p(nn), s6, bp, xp,
                                      _stream(stream)), "ie_nn_predict")


def ie_nn_guess(ctx, nn, sigma6, b, x, stream=None):
    """Learned guess on the full grid; returns 1 (learned), 0 (default kept) or 2 (zero)."""
    s6, bp, xp = _ptrs(_dev_of(ctx), _tensor6(ctx, sigma6), _field(ctx, b, "b"),
                       _field(ctx, x, "x"))
    acc = C.c_int32(0)
    _check(lib().ie_nn_guess(C.c_void_p(ctx), C.c_void_p(nn), s6, bp, xp, C.byref(acc),
                             _stream(stream)), "ie_nn_guess")
    return acc.value
