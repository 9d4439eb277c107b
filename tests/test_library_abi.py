"""Host-side checks of the C-ABI library (no GPU compute): it loads, exports
every function include/fr3d.h declares, and its pure-host entry points behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fr3d.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fr3d_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1703_01216_amd import fr3d
    if not os.path.exists(fr3d.LIB_PATH):
        pytest.fail("libfr3d.so not built (run __graft_entry__.build())")
    return fr3d.lib()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    from paper_1703_01216_amd import fr3d
    assert sorted(fr3d.EXPORTED) == names


def test_every_symbol_resolves_at_load():
    # eager binding: a function the library calls but does not define fails here
    import os
    from paper_1703_01216_amd import fr3d
    ctypes.CDLL(fr3d.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)


def test_defaults_and_status_strings(lib):
    from paper_1703_01216_amd import fr3d
    o = fr3d.default_opts()
    assert (o.log10_alpha_lo, o.log10_alpha_hi, o.max_steps, o.tol) == (-8.0, 0.0, 40, 1e-3)
    assert (o.accept_lo, o.accept_hi, o.tau, o.h_op, o.mu, o.use_predictor) == (0.9, 1.1, 1.0, 0.0, 0.0, 0)
    assert o.seed_walk == 0.25 and o.candidates == 0 and o.seed_slope == 0.0 and o.seed_slope_x == 0.0 and o.seed_snap_lo == 0.0
    assert o.seed_slope_ratio == 0.0
    assert lib.fr3d_status_string(0) == b"ok"
    assert lib.fr3d_status_string(1) == b"invalid argument"
    assert lib.fr3d_last_error(None) == b"null context"


def test_null_arguments_rejected(lib):
    from paper_1703_01216_amd import fr3d
    assert lib.fr3d_create(None, 0, None) == fr3d.E_INVALID
    assert lib.fr3d_destroy(None) == fr3d.E_INVALID
    assert lib.fr3d_set_data(None, None, 0.0) == fr3d.E_INVALID
    assert lib.fr3d_solve_alpha(None, 1.0, None, None) == fr3d.E_INVALID
    # the context-free recovery checks its arguments before touching a device
    one = ctypes.c_void_p(1)
    assert lib.fr3d_recover_c_noalloc(16, 8, one, one, 1.0, one, None, None) == fr3d.E_INVALID
    assert lib.fr3d_recover_c_noalloc(32, -1, one, one, 1.0, one, None, None) == fr3d.E_INVALID
    assert lib.fr3d_recover_c_noalloc(32, (1 << 40) + 1, one, one, 1.0, one, None, None) == fr3d.E_INVALID
    assert lib.fr3d_recover_c_noalloc(64, 8, None, one, 1.0, one, None, None) == fr3d.E_INVALID
    assert lib.fr3d_recover_c_noalloc(64, 8, one, one, 0.0, one, None, None) == fr3d.E_INVALID
    assert lib.fr3d_recover_c_noalloc(64, 8, one, one, float("nan"), one, None, None) == fr3d.E_INVALID


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1703_01216_amd import fr3d
    ctx = ctypes.c_void_p()
    assert lib.fr3d_create(ctypes.byref(ctx), 0, None) == fr3d.E_DEVICE
    assert not ctx.value


def test_struct_layouts_match_header():
    from paper_1703_01216_amd import fr3d
    # int32 x3, (pad) double x2, int32 x3 (+pad)
    assert ctypes.sizeof(fr3d.Geom) == 56 and fr3d.Geom.h.offset == 16 and fr3d.Geom.kind.offset == 32
    assert fr3d.Geom.hz.offset == 48
    assert ctypes.sizeof(fr3d.Report) == 64 and fr3d.Report.n_evals.offset == 40 and fr3d.Report.n_clamped.offset == 48
    assert fr3d.Report.residual_full_box.offset == 56
    assert fr3d.DpOpts.tol.offset == 24 and ctypes.sizeof(fr3d.DpOpts) == 128 and fr3d.DpOpts.seed_walk.offset == 80 and fr3d.DpOpts.seed_slope.offset == 96 and fr3d.DpOpts.seed_snap_lo.offset == 112
    assert fr3d.DpOpts.seed_slope_ratio.offset == 120
    assert fr3d.DpOpts.candidates.offset == 88


def test_ctypes_layouts_equal_c_compiler_layouts(tmp_path):
    # every field offset and struct size of the binding against what a C
    # compiler makes of include/fr3d.h
    import shutil
    import subprocess
    from paper_1703_01216_amd import fr3d
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"fr3d_geom": fr3d.Geom, "fr3d_dp_opts": fr3d.DpOpts, "fr3d_report": fr3d.Report}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "fr3d.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
