"""The C-ABI library loads and exports every entry point its header declares;
host-only argument checks return the documented status codes (no GPU work).
"""
import ctypes
import os
import re

import pytest

from paper_2604_13433_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def declared_symbols():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(pksell_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for n in ("pksell_encode", "pksell_spmv", "pksell_spmv_t", "pksell_pcg"):
        assert n in names, n


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    # every declared entry point also has a Python prototype
    assert set(declared_symbols()) <= set(B.exported_symbols())


def test_version_and_status_strings():
    lib = B.lib()
    assert lib.pksell_version() >= 100
    assert lib.pksell_status_string(0) == b"ok"
    assert lib.pksell_status_string(-1) == b"invalid argument"
    assert lib.pksell_status_string(-5) == b"solver did not converge"


def _query(n=100, m=100, nnz=500, C=64, sigma=256, D=15, fmt=B.FP16, mode=B.IMPLICIT):
    desc = B.CMatrix()
    ws = ctypes.c_size_t()
    rc = B.lib().pksell_encode_query(n, m, nnz, C, sigma, D, fmt, mode, ctypes.byref(desc),
                                     ctypes.byref(ws))
    return rc, desc, ws.value


def test_encode_query_sizes():
    rc, d, ws = _query(n=1000, C=32, sigma=256)
    assert rc == 0 and d.n_slices == 32 and d.perm_bytes == 1 and ws > 0
    rc, d, ws = _query(n=1000, C=64, sigma=4096)
    assert rc == 0 and d.n_slices == 16 and d.perm_bytes == 2


@pytest.mark.parametrize("kw,code", [
    (dict(C=3), B.EINVAL), (dict(C=128), B.EINVAL), (dict(C=0), B.EINVAL),
    (dict(sigma=0), B.EINVAL), (dict(sigma=65537), B.EINVAL),
    (dict(fmt=B.FP16, D=14), B.EINVAL), (dict(fmt=B.E8MY, D=0), B.EINVAL),
    (dict(fmt=B.E8MY, D=23), B.EINVAL), (dict(fmt=B.FIX, D=30), B.EINVAL),
    (dict(fmt=B.E11MY, D=52), B.EINVAL), (dict(fmt=B.E11MY, D=0), B.EINVAL),
    (dict(fmt=7), B.EINVAL), (dict(mode=3), B.EINVAL), (dict(n=-1), B.EINVAL),
    (dict(n=1 << 30), B.ERANGE), (dict(m=1 << 30), B.ERANGE),
])
def test_encode_query_rejects(kw, code):
    rc, _, _ = _query(**kw)
    assert rc == code
    assert B.lib().pksell_last_error()


def test_sell_query_dtypes():
    """float32, float64 and half values are accepted; anything else is not."""
    desc = B.CSell()
    ws = ctypes.c_size_t()
    for dt in (B.F32, B.F64, B.F16):
        rc = B.lib().pksell_sell_query(10, 10, 10, 64, 256, dt, B.IMPLICIT, ctypes.byref(desc),
                                       ctypes.byref(ws))
        assert rc == B.OK and desc.dtype == dt
    for dt in (0, 1, 3, 16):
        rc = B.lib().pksell_sell_query(10, 10, 10, 64, 256, dt, B.IMPLICIT, ctypes.byref(desc),
                                       ctypes.byref(ws))
        assert rc == B.EINVAL


@pytest.mark.parametrize("C,J", [(64, 12), (64, 4), (64, 1 << 25), (32, 64), (64, -8)])
def test_encode_rejects_bad_split_words(C, J):
    """The split check runs on the host before any device work, so dummy
    host buffers stand in for the device arrays."""
    rc, desc, ws = _query(n=100, C=C)
    assert rc == 0
    desc.split_words = J
    buf = (ctypes.c_uint8 * max(ws, 4096))()
    p = ctypes.cast(buf, ctypes.c_void_p)
    desc.offset = p
    desc.perm = p
    rc = B.lib().pksell_encode(p, p, p, B.F32, ctypes.byref(desc), p, max(ws, 4096), None)
    assert rc == B.EINVAL
    assert b"split_words" in B.lib().pksell_last_error()


@pytest.mark.parametrize("n,m,nnz,code", [(-1, 5, 5, B.EINVAL), (5, 5, -2, B.EINVAL),
                                          (1 << 30, 5, 5, B.ERANGE), (5, 5, 1 << 31, B.ERANGE)])
def test_csr_transpose_query_rejects(n, m, nnz, code):
    ws = ctypes.c_size_t()
    assert B.lib().pksell_csr_transpose_query(n, m, nnz, ctypes.byref(ws)) == code
    assert B.lib().pksell_last_error()


def test_stream_read_rejects_on_host():
    buf = (ctypes.c_uint8 * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    for nbytes, width, chunks in [(20, 4, 7), (0, 4, 7), (64, 8, 7), (64, 4, 0), (64, 4, 5000)]:
        assert B.lib().pksell_stream_read(p, nbytes, width, chunks, p, None) == B.EINVAL


def test_encode_rejects_small_workspace():
    rc, desc, ws = _query(n=100)
    assert rc == 0 and ws > 0
    buf = (ctypes.c_uint8 * max(ws, 4096))()
    p = ctypes.cast(buf, ctypes.c_void_p)
    desc.offset = p
    desc.perm = p
    rc = B.lib().pksell_encode(p, p, p, B.F32, ctypes.byref(desc), p, ws - 1, None)
    assert rc == B.EWORKSPACE
    assert b"workspace" in B.lib().pksell_last_error()


def test_encode_query_accepts_e11my_range():
    for D in (1, 15, 51):
        rc, d, ws = _query(fmt=B.E11MY, D=D)
        assert rc == B.OK and d.fmt == B.E11MY and d.D == D


def test_pcg64_rejects_on_host():
    """The 64-bit-word solver checks its outer matrix before any device work:
    a 32-bit-word matrix, a non-square one and explicit row order are
    rejected; dummy host buffers stand in for the device arrays."""
    buf = (ctypes.c_double * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    info = B.CPcgInfo()
    ws = ctypes.c_size_t()
    L = B.lib()
    cases = [dict(fmt=B.E8MY, D=9), dict(fmt=B.E11MY, D=14, m=90),
             dict(fmt=B.E11MY, D=14, mode=B.EXPLICIT)]
    for kw in cases:
        rc, desc, _ = _query(**kw)
        assert rc == B.OK
        desc.offset = desc.perm = desc.pack = p
        rc = L.pksell_pcg64(None, ctypes.byref(desc), p, p, 1e-8, 5, 5, ctypes.byref(info), p,
                            512, None)
        assert rc == B.EINVAL, kw
        assert L.pksell_last_error()
    rc, desc, _ = _query(fmt=B.E8MY, D=9)
    assert L.pksell_pcg64_workspace(None, ctypes.byref(desc), ctypes.byref(ws)) == B.EINVAL


def test_encode_query_16_bit_words():
    """E5MY takes 1 <= D <= 8, FIX16 1 <= D <= 13, both only with C = 64."""
    for fmt, lo, hi in ((B.E5MY, 1, 8), (B.FIX16, 1, 13)):
        for D in (lo, hi):
            rc, d, _ = _query(fmt=fmt, D=D, C=64)
            assert rc == B.OK and d.fmt == fmt and d.D == D
        for D in (lo - 1, hi + 1):
            assert _query(fmt=fmt, D=D, C=64)[0] == B.EINVAL
        assert _query(fmt=fmt, D=lo, C=32)[0] == B.EINVAL


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes struct of the binding has the C struct's size and field
    offsets, read from a program compiled against include/pksell.h (a
    mismatch would hand the library shifted pointers)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"pksell_matrix": B.CMatrix, "pksell_sell": B.CSell, "pksell_batch": B.CBatch,
               "pksell_batch_item": B.CBatchItem, "pksell_pcg_info": B.CPcgInfo}
    rename = {"inp": "in"}  # a Python keyword in the binding
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pksell.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            cf = rename.get(f, f)
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", HEADER_DIR, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_trsv_rejects_on_host():
    """The triangular solves check their arguments before any device work:
    a C = 64 matrix, a non-square one and a level pointer that does not span
    the rows are rejected; an empty schedule needs no device."""
    buf = (ctypes.c_double * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    L = B.lib()
    lp = (ctypes.c_int64 * 3)(0, 2, 3)
    for kw, levels in ((dict(fmt=B.FP16, D=15), 2), (dict(fmt=B.FP16, D=15, C=1, sigma=1, m=4), 2),
                       (dict(fmt=B.FP16, D=15, C=1, sigma=1), 1)):
        rc, desc, _ = _query(n=3, m=kw.pop("m", 3), **kw)
        assert rc == B.OK
        desc.offset = desc.pack = p
        rc = L.pksell_trsv(ctypes.byref(desc), 0, p, ctypes.cast(lp, ctypes.c_void_p), levels, p,
                           p, None)
        assert rc == B.EINVAL, kw
        assert L.pksell_last_error()
    assert L.pksell_trsv_csr(p, p, p, 3, 0, p, ctypes.cast(lp, ctypes.c_void_p), 1, p, p,
                             None) == B.EINVAL
    nl = ctypes.c_int64(7)
    lp0 = (ctypes.c_int64 * 1)(5)
    assert L.pksell_trsv_levels(None, None, 0, 0, None, ctypes.cast(lp0, ctypes.c_void_p),
                                ctypes.byref(nl), None) == B.OK
    assert nl.value == 0 and lp0[0] == 0
    assert L.pksell_trsv_levels(None, None, -1, 1, None, ctypes.cast(lp0, ctypes.c_void_p),
                                ctypes.byref(nl), None) == B.ERANGE


@pytest.mark.parametrize("sigma,J", [(2, 512), (1, 384), (1, 2048), (1, 128)])
def test_encode_checks_chunk_words_for_one_row_slices(sigma, J):
    """C = 1 takes split_words as the chunk size of the balanced product:
    256, 512 or 1024 words, and only with sigma = 1 (the GPU tests build
    the valid ones).  The check runs on the host before any device work
    (dummy host buffers stand in)."""
    rc, desc, ws = _query(n=100, C=1, sigma=sigma, mode=B.EXPLICIT)
    assert rc == 0
    desc.split_words = J
    buf = (ctypes.c_uint8 * max(ws, 4096))()
    p = ctypes.cast(buf, ctypes.c_void_p)
    desc.offset = p
    rc = B.lib().pksell_encode(p, p, p, B.F32, ctypes.byref(desc), p, max(ws, 4096), None)
    assert rc == B.EINVAL
    assert b"split_words" in B.lib().pksell_last_error()


@pytest.mark.parametrize("n,m,nnz,T", [(10, 10, 10, 300), (10, 10, 10, 128), (-1, 10, 10, 512),
                                       (1 << 30, 10, 10, 512), (10, 10, 1 << 31, 512)])
def test_csr32_query_rejects(n, m, nnz, T):
    d = B.CCsr32()
    assert B.lib().pksell_csr32_query(n, m, nnz, T, ctypes.byref(d)) == B.EINVAL
    assert B.lib().pksell_last_error()


def test_csr32_query_sizes():
    d = B.CCsr32()
    assert B.lib().pksell_csr32_query(7, 9, 1025, 512, ctypes.byref(d)) == B.OK
    assert (d.n, d.m, d.nnz, d.T, d.n_chunks) == (7, 9, 1025, 512, 3)
    assert ctypes.sizeof(B.CCsr32) == 72
