"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/mts.h declares, its structs match the binding's
layout, and invalid arguments are rejected before any HIP call."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_2208_01525_amd as P
from paper_2208_01525_amd import mts as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mts_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = P.load()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(M.EXPORTS)
    nm = subprocess.run(["nm", "-D", M.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (mts_\w+)", nm))
    assert set(names) <= exported


def test_struct_layout_matches_header():
    """Compile a probe against include/mts.h with the host compiler and compare
    sizeof/offsetof with the ctypes mirrors."""
    fields_p = [f for f, _ in M.Params._fields_]
    fields_d = [f for f, _ in M.Diag._fields_]
    fields_s = [f for f, _ in M.Segments._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "mts.h"', "int main(void){"]
    src.append('printf("%zu %zu %zu\\n", sizeof(mts_params), sizeof(mts_diag), sizeof(mts_segments_t));')
    for f in fields_p:
        src.append(f'printf("%zu\\n", offsetof(mts_params, {f}));')
    for f in fields_d:
        src.append(f'printf("%zu\\n", offsetof(mts_diag, {f}));')
    for f in fields_s:
        src.append(f'printf("%zu\\n", offsetof(mts_segments_t, {f}));')
    src.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write("\n".join(src))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(M.Params) and vals[1] == ctypes.sizeof(M.Diag)
    assert vals[2] == ctypes.sizeof(M.Segments)
    offs = vals[3:]
    np_, nd = len(fields_p), len(fields_d)
    assert offs[:np_] == [getattr(M.Params, f).offset for f in fields_p]
    assert offs[np_:np_ + nd] == [getattr(M.Diag, f).offset for f in fields_d]
    assert offs[np_ + nd:] == [getattr(M.Segments, f).offset for f in fields_s]


def test_state_bytes():
    """30 planes of the site count rounded up to 64 elements, each followed by a 4 KiB
    stagger."""
    p = P.make_params(64, eta_ref=17.0)
    assert P.state_bytes(p) == 30 * (64 ** 3 * 4 + 4096)
    p = P.make_params(5, 6, 7, precision="fp64")
    assert P.state_bytes(p) == 30 * (256 * 8 + 4096)          # 210 sites rounded up to 256
    p512 = P.make_params(512, eta_ref=128.0)
    assert P.state_bytes(p512) == 30 * (512 ** 3 * 4 + 4096)  # 16.1 GB: fits one MI355X


@pytest.mark.parametrize("field,value", [
    ("nx", 3), ("nz", 0), ("precision", 3), ("dx", 0.0), ("dt", -0.1), ("e_p", 0.0), ("sigma_q", -1.0),
    ("lambda_p", -2.0), ("eta_ref", 0.0), ("diag_every", -1), ("overlap_radius", 2), ("kappa", float("nan")),
])
def test_invalid_params_rejected_without_gpu(field, value):
    p = P.make_params(8, eta_ref=4.0)
    setattr(p, field, value)
    assert P.state_bytes(p) == 0
    out = ctypes.c_void_p()
    rc = P.load().mts_create(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(out))
    assert rc == M.MTS_EINVAL and not out.value


def test_too_large_box_rejected():
    """Planes are indexed with 32 bits: the site count plus the plane stagger must fit."""
    p = P.make_params(2048, 2048, 1024, eta_ref=4.0)     # 2^32 sites
    assert P.state_bytes(p) == 0
    p = P.make_params(4, 4, 268435392, eta_ref=4.0)      # 2^32 - 1024 sites: the stagger would overflow
    assert 4 * 4 * 268435392 == 2 ** 32 - 1024
    assert P.state_bytes(p) == 0
    p = P.make_params(2048, 2048, 1023, eta_ref=4.0)     # just below: accepted
    assert P.state_bytes(p) == 30 * ((2048 * 2048 * 1023) * 4 + 4096)


def test_create_checks_buffer_before_gpu():
    L = P.load()
    p = P.make_params(8, eta_ref=4.0)
    out = ctypes.c_void_p()
    assert L.mts_create(ctypes.byref(p), None, 1 << 20, None, ctypes.byref(out)) == M.MTS_EINVAL
    assert L.mts_create(ctypes.byref(p), ctypes.c_void_p(256 + 8), 1 << 20, None, ctypes.byref(out)) == M.MTS_EINVAL
    assert L.mts_create(ctypes.byref(p), ctypes.c_void_p(256), 100, None, ctypes.byref(out)) == M.MTS_ENOMEM


def test_null_context_rejected():
    L = P.load()
    assert L.mts_step(None, 1, 1.0, 0.5, 1.0) == M.MTS_EINVAL
    assert L.mts_init_fields(None, 1) == M.MTS_EINVAL
    cnt = ctypes.c_int32()
    assert L.mts_diagnostics(None, None, 0, ctypes.byref(cnt)) == M.MTS_EINVAL
    assert L.mts_strerror(M.MTS_EUNSTABLE) == b"MTS_EUNSTABLE"
    assert L.mts_autotune_cached(None, 3, b"/nonexistent/cache", None, None, None, None) == M.MTS_EINVAL
    assert L.mts_batch_set_persistent(None, 1, 0.0) == M.MTS_EINVAL


def test_noalloc_limit_matches_header_and_null_context_rejected():
    text = open(HEADER).read()
    m = re.search(r"#define MTS_NOALLOC_MAX_SITES (\d+)", text)
    assert m and int(m.group(1)) == M.NOALLOC_MAX_SITES
    L = P.load()
    out = (ctypes.c_double * 20)()
    site = (ctypes.c_uint64 * 1)(0)
    assert L.mts_get_sites_noalloc(None, site, 1, out) == M.MTS_EINVAL
