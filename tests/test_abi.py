"""The C-ABI library: it loads, exports every symbol include/ie.h declares, its ctypes
structures match the C layout, and host-side validation rejects bad input before any GPU work
(none of these tests launches a kernel)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ie.h")


@pytest.fixture(scope="module")
def L():
    from paper_2306_17537_amd import ie
    if not os.path.exists(ie.LIB_PATH):
        from paper_2306_17537_amd import build_lib
        build_lib.build(verbose=False)
    return ie


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(ie_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert {"ie_green_setup", "ie_matvec", "ie_gmres", "ie_dd_solve"} <= set(names)
    lib = C.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True)
    exported = set(re.findall(r"\bT (ie_\w+)", out.stdout))
    assert set(names) <= exported


def test_struct_layout_matches_c(L, tmp_path):
    """Compile a C probe of sizeof/offsetof against ie.h and compare with the ctypes mirrors."""
    structs = {
        "ie_grid": L.ie_grid, "ie_medium": L.ie_medium, "ie_source": L.ie_source,
        "ie_partition": L.ie_partition, "ie_gmres_opts": L.ie_gmres_opts,
        "ie_gmres_stats": L.ie_gmres_stats, "ie_dd_opts": L.ie_dd_opts,
        "ie_dd_stats": L.ie_dd_stats, "ie_problem": L.ie_problem,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ie.h"', "int main(void){"]
    for s, cls in structs.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                         text=True).stdout.split("\n") if l)
    for s, cls in structs.items():
        assert int(got[s]) == C.sizeof(cls), s
        for f, _ in cls._fields_:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, f"{s}.{f}"


def test_version_and_error_string(L):
    assert L.ie_version().startswith("ie-gfx950")
    assert isinstance(L.ie_last_error(), str)


@pytest.mark.parametrize("n,h,sig,f,zb,msg", [
    ((0, 4, 4), 0.25, 0.1, 1e5, None, "grid size"),
    ((4, 4, 600), 0.25, 0.1, 1e5, None, "grid size"),
    ((4, 4, 4), -1.0, 0.1, 1e5, None, "cell size"),
    ((4, 4, 4), 0.25, 0.0, 1e5, None, "sigma0"),
    ((4, 4, 4), 0.25, 0.1, -2.0, None, "frequency"),
    ((4, 4, 4), 0.25, 0.1, 1e5, (0, 2, 3), "end at nz"),
    ((4, 4, 4), 0.25, 0.1, 1e5, (0, 2, 2, 4), "increase"),
    ((4, 4, 4), 0.25, 0.1, 1e5, (1, 4), "start at 0"),
])
def test_setup_rejects_bad_input_on_host(L, n, h, sig, f, zb, msg):
    g = L.make_grid(n, h, (0.0, 0.0, 0.0))
    m = L.ie_medium(sig, f, 0.0)
    part = None
    if zb is not None:
        arr = (C.c_int32 * len(zb))(*zb)
        part = L.ie_partition(len(zb) - 1, arr)
    out = C.c_void_p(123)
    rc = L.lib().ie_green_setup(C.byref(g), C.byref(m), C.byref(part) if part else None,
                                L.IE_FP64, None, C.byref(out))
    assert rc == L.IE_EINVAL
    assert out.value is None
    assert msg in L.ie_last_error()


def test_entry_points_reject_null_arguments(L):
    lib = L.lib()
    assert lib.ie_matvec(None, None, None, None, 0, 1, None) == L.IE_EINVAL
    assert lib.ie_gmres(None, None, None, None, None, None, None) == L.IE_EINVAL
    assert lib.ie_dd_solve(None, 0, None, None, None, None) == L.IE_EINVAL
    assert lib.ie_background_field(None, None, 0, None, None) == L.IE_EINVAL
    assert lib.ie_ctx_destroy(None) == L.IE_OK


def test_set_option_validates_on_host(L):
    lib = L.lib()
    for opt, bad in ((L.IE_OPT_GRAPHS, 2), (L.IE_OPT_AUTOTUNE, -1), (L.IE_OPT_FORCE_VARIANT, 8),
                     (L.IE_OPT_GROUP_THREADS, 2), (99, 0)):
        assert lib.ie_set_option(opt, bad) == L.IE_EINVAL, (opt, bad)
    for opt, good, default in ((L.IE_OPT_GRAPHS, 0, 1), (L.IE_OPT_GROUP_THREADS, 0, 1),
                               (L.IE_OPT_FORCE_VARIANT, 3, -1)):
        assert lib.ie_set_option(opt, good) == L.IE_OK
        assert lib.ie_set_option(opt, default) == L.IE_OK
