"""Thin Python binding of ``libpksell.so`` (the C ABI in include/pksell.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's
kernels.  There is no fallback: if the library is missing, loading it
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpksell.so")

OK, EINVAL, ERANGE, EWORKSPACE, EHIP, ENOTCONV, EBREAKDOWN = 0, -1, -2, -3, -4, -5, -6
FP16, E8MY, FIX, E11MY, E5MY, FIX16 = 0, 1, 2, 3, 4, 5  # E5MY, FIX16: 16-bit words
EXPLICIT, IMPLICIT = 0, 1
F32, F64, F16 = 4, 8, 2  # F16: SELL half values (float32 vectors)
F32_PAIRED = 12  # SELL float32 values and int32 columns in one 8-byte slot
CACHE_STREAM, CACHE_RESIDENT = 0, 1  # cache_hint of a matrix (include/pksell.h)
FMT_BY_NAME = {"fp16": FP16, "e8my": E8MY, "fix": FIX, "e11my": E11MY, "e5my": E5MY,
               "fix16": FIX16}
W16 = (E5MY, FIX16)

i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p


class PackSELLError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"pksell error {status}: {detail}")
        self.status = status


class CMatrix(ctypes.Structure):
    _fields_ = [("n", i64), ("m", i64), ("nnz", i64),
                ("C", i32), ("sigma", i32), ("D", i32), ("fmt", i32),
                ("perm_mode", i32), ("perm_bytes", i32),
                ("n_slices", i64), ("n_words", i64), ("n_dummies", i64), ("k_left", i64),
                ("pack", vp), ("offset", vp), ("perm", vp), ("row_exp", vp),
                ("split_words", i32), ("cache_hint", i32),
                ("n_units", i64), ("n_split_units", i64), ("n_split_slices", i64),
                ("units", vp), ("splits", vp), ("ckpt", vp), ("partial", vp)]


class CSell(ctypes.Structure):
    _fields_ = [("n", i64), ("m", i64), ("nnz", i64),
                ("C", i32), ("sigma", i32), ("perm_mode", i32), ("perm_bytes", i32),
                ("dtype", i32), ("cache_hint", i32),
                ("n_slices", i64), ("n_slots", i64),
                ("offset", vp), ("perm", vp), ("col", vp), ("val", vp)]


class CBatchItem(ctypes.Structure):
    _fields_ = [("A", ctypes.POINTER(CMatrix)), ("inp", vp), ("out", vp)]


class CBatch(ctypes.Structure):
    _fields_ = [("count", i32), ("fmt", i32), ("k", i32), ("transpose", i32),
                ("total_units", i64), ("units_per_wave", i32), ("waves", i32),
                ("vec4", i32), ("group", i32), ("words_per_group", i32), ("pair_units", i32),
                ("items", vp), ("unit_start", vp)]


class CCsr32(ctypes.Structure):
    _fields_ = [("n", i64), ("m", i64), ("nnz", i64), ("T", i32), ("reserved", i32),
                ("n_chunks", i64), ("rowptr", vp), ("ent", vp), ("lo", vp), ("partial", vp)]


class CF3RParams(ctypes.Structure):
    _fields_ = [("m1", i32), ("m2", i32), ("m3", i32), ("m4", i32), ("omega", ctypes.c_double),
                ("max_cycles", i32), ("reserved", i32)]


class CPcgInfo(ctypes.Structure):
    _fields_ = [("outer_iterations", i32), ("inner_iterations", i32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


_lib = None

_PROTOS = {
    "pksell_version": ([], ctypes.c_int),
    "pksell_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "pksell_last_error": ([], ctypes.c_char_p),
    "pksell_encode_query": ([i64, i64, i64, i32, i32, i32, i32, i32,
                             ctypes.POINTER(CMatrix), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pksell_encode": ([vp, vp, vp, i32, ctypes.POINTER(CMatrix), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "pksell_spmv": ([ctypes.POINTER(CMatrix), vp, vp, i64, vp], ctypes.c_int),
    "pksell_spmv_static": ([ctypes.POINTER(CMatrix), vp, vp, i64, vp], ctypes.c_int),
    "pksell_spmv_f64": ([ctypes.POINTER(CMatrix), vp, vp, ctypes.c_int64, vp], ctypes.c_int),
    "pksell_spmv_t": ([ctypes.POINTER(CMatrix), vp, vp, i64, vp], ctypes.c_int),
    "pksell_grad_values": ([ctypes.POINTER(CMatrix), vp, vp, vp, vp, i64, vp], ctypes.c_int),
    "pksell_decode": ([ctypes.POINTER(CMatrix), vp, vp, vp], ctypes.c_int),
    "pksell_sell_query": ([i64, i64, i64, i32, i32, i32, i32,
                           ctypes.POINTER(CSell), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pksell_sell_encode": ([vp, vp, vp, i32, ctypes.POINTER(CSell), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "pksell_sell_spmv": ([ctypes.POINTER(CSell), vp, vp, vp], ctypes.c_int),
}

_PROTOS.update({
    "pksell_csr_transpose_query": ([i64, i64, i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pksell_csr_transpose": ([vp, vp, vp, i32, i64, i64, i64, vp, vp, vp, vp, ctypes.c_size_t, vp],
                             ctypes.c_int),
    "pksell_stream_read": ([vp, ctypes.c_size_t, i32, i32, vp, vp], ctypes.c_int),
    "pksell_trsv_levels": ([vp, vp, i64, i32, vp, vp, ctypes.POINTER(i64), vp], ctypes.c_int),
    "pksell_trsv": ([ctypes.POINTER(CMatrix), i32, vp, vp, i64, vp, vp, vp], ctypes.c_int),
    "pksell_trsv_csr": ([vp, vp, vp, i64, i32, vp, vp, i64, vp, vp, vp], ctypes.c_int),
    "pksell_batch_plan_bytes": ([i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pksell_batch_plan": ([ctypes.POINTER(CBatchItem), i32, i64, i32, ctypes.POINTER(CBatch), vp,
                           ctypes.c_size_t, vp], ctypes.c_int),
    "pksell_spmv_batched": ([ctypes.POINTER(CBatch), vp], ctypes.c_int),
    "pksell_pcg_workspace": ([ctypes.POINTER(CMatrix), ctypes.POINTER(CSell),
                              ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pksell_pcg": ([ctypes.POINTER(CMatrix), ctypes.POINTER(CSell), vp, vp, ctypes.c_double,
                    i32, i32, ctypes.POINTER(CPcgInfo), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "pksell_f3r_workspace": ([i64, i32, ctypes.POINTER(CF3RParams),
                              ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pksell_f3r": ([ctypes.POINTER(CSell), ctypes.POINTER(CSell), ctypes.POINTER(CSell),
                    ctypes.POINTER(CMatrix), vp, vp, ctypes.c_double, ctypes.POINTER(CF3RParams),
                    ctypes.POINTER(CPcgInfo), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "pksell_csr32_query": ([i64, i64, i64, i32, ctypes.POINTER(CCsr32)], ctypes.c_int),
    "pksell_csr32_encode": ([vp, vp, i32, ctypes.POINTER(CCsr32), vp], ctypes.c_int),
    "pksell_csr32_spmv": ([ctypes.POINTER(CCsr32), vp, vp, vp], ctypes.c_int),
    "pksell_pcg64_workspace": ([ctypes.POINTER(CMatrix), ctypes.POINTER(CMatrix),
                                ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pksell_pcg64": ([ctypes.POINTER(CMatrix), ctypes.POINTER(CMatrix), vp, vp, ctypes.c_double,
                      i32, i32, ctypes.POINTER(CPcgInfo), vp, ctypes.c_size_t, vp], ctypes.c_int),
})

OPTIONAL: dict = {}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in {**_PROTOS, **OPTIONAL}.items():
            if hasattr(L, name):
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return sorted(set(_PROTOS) | set(OPTIONAL))


def _check(status: int):
    if status != OK:
        raise PackSELLError(status, lib().pksell_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require(cond: bool, msg: str):
    """Argument check that survives ``python -O`` (unlike assert)."""
    if not cond:
        raise ValueError(msg)


def _block(t, dtype, rows: int, k: int | None, name: str):
    """Checks a dense vector or row-major block argument: dtype, contiguity,
    a GPU tensor, ``rows`` rows and (when given) ``k`` columns."""
    _require(isinstance(t, torch.Tensor), f"{name} must be a torch tensor")
    _require(t.dtype == dtype, f"{name} must be {dtype}, got {t.dtype}")
    _require(t.dim() in (1, 2) and t.shape[0] == rows,
             f"{name} must have {rows} rows, got shape {tuple(t.shape)}")
    if k is not None:
        kk = 1 if t.dim() == 1 else t.shape[1]
        _require(kk == k, f"{name} must have {k} columns, got {kk}")
    _require(t.is_contiguous(), f"{name} must be contiguous")
    _require(t.is_cuda, f"{name} must be a GPU tensor")


def _dev(t, dtype, device):
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    return t.to(device=device, dtype=dtype).contiguous()


# Integer fields of the descriptor (everything but the device pointers).
_DESC_INTS = ("n", "m", "nnz", "C", "sigma", "D", "fmt", "perm_mode", "perm_bytes", "n_slices",
              "n_words", "n_dummies", "k_left", "split_words", "n_units", "n_split_units",
              "n_split_slices")


class PackSELLMatrix:
    """A PackSELL matrix on the GPU (device arrays held as torch tensors)."""

    def __init__(self, desc: CMatrix, tensors: dict, device):
        self.desc = desc
        self.t = tensors
        self.device = device

    # shape / statistics
    n = property(lambda s: s.desc.n)
    m = property(lambda s: s.desc.m)
    nnz = property(lambda s: s.desc.nnz)
    n_words = property(lambda s: s.desc.n_words)
    n_dummies = property(lambda s: s.desc.n_dummies)
    k_left = property(lambda s: s.desc.k_left)
    fmt = property(lambda s: s.desc.fmt)
    D = property(lambda s: s.desc.D)
    C = property(lambda s: s.desc.C)
    sigma = property(lambda s: s.desc.sigma)
    perm_mode = property(lambda s: s.desc.perm_mode)

    @property
    def cache_hint(self) -> int:
        """CACHE_STREAM (the default) or CACHE_RESIDENT: how the
        single-vector product (k = 1, C = 64) loads the words (same results
        either way)."""
        return self.desc.cache_hint

    @cache_hint.setter
    def cache_hint(self, v: int):
        self.desc.cache_hint = int(v)

    @property
    def pack(self):
        return self.t["pack"]

    @property
    def offset(self):
        return self.t["offset"]

    @property
    def perm(self):
        p = self.t.get("perm")
        if p is None:
            return None
        if self.desc.perm_bytes == 1:
            return p.view(torch.uint8)
        return p.view(torch.int16).to(torch.int32) & 0xFFFF  # unsigned 16-bit values

    @property
    def row_exp(self):
        return self.t.get("row_exp")

    def bytes_per_spmv(self, k: int = 1) -> int:
        """Algorithmic bytes of one product: every stored word (padding and
        dummies included), the offsets, perm (implicit), row exponents
        (FIX), x once and y once."""
        d = self.desc
        if d.fmt == E11MY:  # 8-byte words, float64 x and y
            b = 8 * d.n_words + 8 * (d.n_slices + 1) + 8 * d.m * k + 8 * d.n * k
            if d.perm_mode == IMPLICIT:
                b += d.perm_bytes * d.n
            return int(b)
        wb = 2 if d.fmt in W16 else 4  # bytes per word
        b = wb * d.n_words + 8 * (d.n_slices + 1) + 4 * d.m * k + 4 * d.n * k
        chunked = d.C == 1 and d.split_words > 0 and k in (1, 2, 4)
        if d.perm_mode == IMPLICIT and not chunked:  # rows stay in order: no perm read
            b += d.perm_bytes * d.n
        if d.fmt in (FIX, FIX16):
            b += 2 * d.n
        if chunked and d.n_units > 0:
            b += 12 * d.n_units + 4  # chunk plan read, each chunk's row marker written
        return int(b)

    def replicate(self):
        """A copy with its own word/offset/perm arrays (same descriptor)."""
        t = {k: v.clone() for k, v in self.t.items()}
        desc = CMatrix.from_buffer_copy(self.desc)
        m = PackSELLMatrix(desc, t, self.device)
        m._bind()
        return m

    def _bind(self):
        d = self.desc
        d.pack = self.t["pack"].data_ptr() if self.t.get("pack") is not None else None
        d.offset = self.t["offset"].data_ptr()
        d.perm = self.t["perm"].data_ptr() if self.t.get("perm") is not None else None
        d.row_exp = self.t["row_exp"].data_ptr() if self.t.get("row_exp") is not None else None
        for name in ("units", "splits", "ckpt", "partial"):
            v = self.t.get(name)
            setattr(d, name, v.data_ptr() if v is not None else None)

    def save(self, path: str):
        """Writes the descriptor and every device array to an .npz file (no
        pickles: plain arrays and integers)."""
        d = self.desc
        meta = {f: int(getattr(d, f)) for f in _DESC_INTS}
        arrays = {k: v.cpu().numpy() for k, v in self.t.items()}
        np.savez(path, **{f"meta_{k}": np.int64(v) for k, v in meta.items()},
                 **{f"arr_{k}": v for k, v in arrays.items()})

    @classmethod
    def load(cls, path: str, device="cuda") -> "PackSELLMatrix":
        """Reads a matrix written by ``save`` onto ``device``."""
        device = torch.device(device)
        with np.load(path, allow_pickle=False) as z:
            desc = CMatrix()
            for f in _DESC_INTS:
                setattr(desc, f, int(z[f"meta_{f}"]))
            t = {k[4:]: torch.from_numpy(z[k]).to(device) for k in z.files if k.startswith("arr_")}
        m = cls(desc, t, device)
        m._bind()
        return m

    @property
    def split_words(self) -> int:
        return self.desc.split_words

    @property
    def n_units(self) -> int:
        return self.desc.n_units

    @property
    def n_split_units(self) -> int:
        return self.desc.n_split_units

    @property
    def n_split_slices(self) -> int:
        return self.desc.n_split_slices


def encode(rowptr, col, val, n: int, m: int, fmt="fp16", D: int = 15, C: int = 64,
           sigma: int = 256, perm_mode: int = IMPLICIT, device="cuda",
           keep_perm: bool = True, analyse_only: bool = False,
           split_words: int = 0) -> PackSELLMatrix:
    """CSR (numpy or torch; values float32 or float64) -> PackSELL on the GPU.
    With ``analyse_only`` only the analyse phase runs: the descriptor then
    holds n_words, n_dummies, k_left and the work-unit counts, and no words
    are written.  ``split_words`` = J > 0 (C = 64, a multiple of 8) splits
    slices wider than J words per lane into chunks of J words for the
    single-vector product; with C = 1 and sigma = 1 (CSR-packed: every
    row's words together, no padding) J = 256, 512 or 1024 cuts the word
    stream into chunks of J words for a product balanced over words."""
    if isinstance(fmt, str):
        fmt = FMT_BY_NAME[fmt]
    device = torch.device(device)
    rp = _dev(rowptr, torch.int64, device)
    cl = _dev(col, torch.int32, device)
    if isinstance(val, np.ndarray):
        vdt = torch.float64 if val.dtype == np.float64 else torch.float32
    else:
        vdt = torch.float64 if val.dtype == torch.float64 else torch.float32
    vl = _dev(val, vdt, device)
    nnz = int(cl.numel())
    desc = CMatrix()
    ws_bytes = ctypes.c_size_t()
    L = lib()
    _check(L.pksell_encode_query(n, m, nnz, C, sigma, D, fmt, perm_mode,
                                 ctypes.byref(desc), ctypes.byref(ws_bytes)))
    desc.split_words = int(split_words)
    t = {"offset": torch.empty(desc.n_slices + 1, dtype=torch.int64, device=device)}
    if perm_mode == IMPLICIT or keep_perm:
        t["perm"] = torch.empty(max(1, n * desc.perm_bytes), dtype=torch.uint8, device=device)
    ws = torch.empty(max(1, ws_bytes.value), dtype=torch.uint8, device=device)
    A = PackSELLMatrix(desc, t, device)
    A._bind()
    st = _stream(device)
    vcode = F64 if vdt == torch.float64 else F32
    _check(L.pksell_encode(_ptr(rp), _ptr(cl), _ptr(vl), vcode, ctypes.byref(desc),
                           _ptr(ws), ws_bytes.value, st))
    if analyse_only:
        return A
    if fmt == E11MY:  # 64-bit words
        t["pack"] = torch.empty(max(1, desc.n_words), dtype=torch.int64, device=device)
    elif fmt in W16:  # 16-bit words, two per 32-bit slot
        t["pack"] = torch.empty(max(1, desc.n_words // 2), dtype=torch.int32, device=device)
    else:
        t["pack"] = torch.empty(max(1, desc.n_words), dtype=torch.int32, device=device)
    if fmt in (FIX, FIX16):
        t["row_exp"] = torch.empty(max(1, n), dtype=torch.int16, device=device)
    if desc.C == 1 and desc.split_words > 0 and desc.n_units > 0:  # CSR-packed chunk plan
        t["units"] = torch.empty(desc.n_units + 1, dtype=torch.int32, device=device)
        t["ckpt"] = torch.empty(desc.n_units, dtype=torch.int32, device=device)
        t["partial"] = torch.empty(9 * desc.n_units, dtype=torch.float32, device=device)
    if desc.n_split_units > 0:
        t["units"] = torch.empty(4 * desc.n_units, dtype=torch.int32, device=device)
        t["splits"] = torch.empty(4 * desc.n_split_slices, dtype=torch.int32, device=device)
        t["ckpt"] = torch.empty(64 * desc.n_split_units, dtype=torch.int32, device=device)
        t["partial"] = torch.empty(64 * desc.n_split_units, dtype=torch.float32, device=device)
    A._bind()
    _check(L.pksell_encode(_ptr(rp), _ptr(cl), _ptr(vl), vcode, ctypes.byref(desc),
                           _ptr(ws), ws_bytes.value, st))
    return A


def encode_packed_csr(rowptr, col, val, n: int, m: int, fmt="fp16", D: int = 15,
                      chunk: int = 512, device="cuda") -> PackSELLMatrix:
    """CSR-based delta-value packing: PackSELL words of each row stored
    together in row order (one-row slices, no sort, no padding), with the
    plan of a product balanced over chunks of ``chunk`` words."""
    return encode(rowptr, col, val, n, m, fmt, D, 1, 1, EXPLICIT, device, split_words=chunk)


class TriangularSolve:
    """y = L_q^{-1} b for a triangular L: lower with every row ending in its
    diagonal, or (``upper``) upper with every row starting with it.  The
    CSR-packed words of L (FP16, E8MY or FIX) and its level schedule are
    built once; each call launches one kernel per level.  With ``fmt=None``
    the solve runs on plain CSR (float32 values, int32 columns) instead,
    the comparator."""

    def __init__(self, rowptr, col, val, n: int, fmt="fp16", D: int = 15, device="cuda",
                 upper: bool = False):
        device = torch.device(device)
        self.n, self.device, self.upper = n, device, int(bool(upper))
        self.rp = _dev(rowptr, torch.int64, device)
        self.cl = _dev(col, torch.int32, device)
        self.order = torch.empty(max(1, n), dtype=torch.int32, device=device)
        self.level_ptr = np.zeros(n + 1, dtype=np.int64)
        nl = i64()
        _check(lib().pksell_trsv_levels(_ptr(self.rp), _ptr(self.cl), n, self.upper,
                                        _ptr(self.order),
                                        self.level_ptr.ctypes.data_as(vp), ctypes.byref(nl),
                                        _stream(device)))
        self.n_levels = int(nl.value)
        self.fmt = fmt
        if fmt is None:
            self.val = _dev(val, torch.float32, device)
            self.L = None
        else:
            self.L = encode(rowptr, col, val, n, n, fmt, D, 1, 1, EXPLICIT, device)

    def bytes_per_solve(self) -> int:
        """Algorithmic bytes: the stored words (or 8 B per CSR entry), the
        row pointer, the schedule, b once, y written once and y gathered
        once per off-diagonal entry at 4 B."""
        nnz = int(self.cl.numel())
        stored = 4 * self.L.n_words if self.L is not None else 8 * nnz
        return int(stored + 8 * (self.n + 1) + 4 * self.n + 8 * self.n + 4 * (nnz - self.n))

    def __call__(self, b: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        _block(b, torch.float32, self.n, 1, "b")
        _require(b.dim() == 1, "b must be a vector")
        if y is None:
            y = torch.empty(self.n, dtype=torch.float32, device=b.device)
        _block(y, torch.float32, self.n, 1, "y")
        _require(y.data_ptr() != b.data_ptr() or self.n == 0, "y must not alias b")
        lp = self.level_ptr.ctypes.data_as(vp)
        if self.L is None:
            _check(lib().pksell_trsv_csr(_ptr(self.rp), _ptr(self.cl), _ptr(self.val), self.n,
                                         self.upper, _ptr(self.order), lp, self.n_levels,
                                         _ptr(b), _ptr(y), _stream(b.device)))
        else:
            _check(lib().pksell_trsv(ctypes.byref(self.L.desc), self.upper, _ptr(self.order),
                                     lp, self.n_levels, _ptr(b), _ptr(y), _stream(b.device)))
        return y


class StreamRead:
    """One streaming read of ``buf`` (a device tensor whose byte size is a
    multiple of 16) per call: the HBM read ceiling for that transfer size.
    ``width`` (4 or 16) bytes per lane and load, ``chunks`` wave-wide pieces
    per wave."""

    def __init__(self, buf: torch.Tensor, width: int = 4, chunks: int = 7):
        _require(buf.is_cuda and buf.is_contiguous() and buf.data_ptr() % 16 == 0,
                 "buf must be a contiguous, 16-byte aligned GPU tensor")
        self.buf = buf
        self.bytes = buf.numel() * buf.element_size()
        self.width, self.chunks = width, chunks
        self.out = torch.empty(1, dtype=torch.float32, device=buf.device)

    def __call__(self):
        _check(lib().pksell_stream_read(_ptr(self.buf), self.bytes, self.width, self.chunks,
                                        _ptr(self.out), _stream(self.buf.device)))


def csr_transpose(rowptr, col, val, n: int, m: int, device="cuda"):
    """CSR of A^T on the device: (t_rowptr int64[m+1], t_col int32[nnz],
    t_val[nnz]) with t_val in val's float type."""
    device = torch.device(device)
    rp = _dev(rowptr, torch.int64, device)
    cl = _dev(col, torch.int32, device)
    f64 = (isinstance(val, np.ndarray) and val.dtype == np.float64) or \
        (isinstance(val, torch.Tensor) and val.dtype == torch.float64)
    vl = _dev(val, torch.float64 if f64 else torch.float32, device)
    nnz = int(cl.numel())
    ws_bytes = ctypes.c_size_t()
    _check(lib().pksell_csr_transpose_query(n, m, nnz, ctypes.byref(ws_bytes)))
    ws = torch.empty(max(1, ws_bytes.value), dtype=torch.uint8, device=device)
    t_rowptr = torch.empty(m + 1, dtype=torch.int64, device=device)
    t_col = torch.empty(max(1, nnz), dtype=torch.int32, device=device)
    t_val = torch.empty(max(1, nnz), dtype=vl.dtype, device=device)
    _check(lib().pksell_csr_transpose(_ptr(rp), _ptr(cl), _ptr(vl), F64 if f64 else F32, n, m, nnz,
                                      _ptr(t_rowptr), _ptr(t_col), _ptr(t_val), _ptr(ws),
                                      ws_bytes.value, _stream(device)))
    return t_rowptr, t_col[:nnz], t_val[:nnz]


def encode_transpose(rowptr, col, val, n: int, m: int, fmt="fp16", D: int = 15, C: int = 64,
                     sigma: int = 256, perm_mode: int = IMPLICIT, device="cuda",
                     split_words: int = 0) -> PackSELLMatrix:
    """PackSELL of A^T (m x n) from the CSR of A, transposed on the device.
    For FP16 and E8MY it holds exactly (A_q)^T, so ``spmv`` on it is the
    adjoint product A_q^T g."""
    if isinstance(fmt, str):
        fmt = FMT_BY_NAME[fmt]
    if fmt in (FIX, FIX16):
        raise ValueError("FIX quantises per row: a transposed copy would not hold (A_q)^T")
    t_rowptr, t_col, t_val = csr_transpose(rowptr, col, val, n, m, device)
    return encode(t_rowptr, t_col, t_val, m, n, fmt, D, C, sigma, perm_mode, device,
                  split_words=split_words)


def spmv(A: PackSELLMatrix, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """y = A_q x (x: m or m x k float32 on the device)."""
    _block(x, torch.float32, A.m, None, "x")
    k = 1 if x.dim() == 1 else x.shape[1]
    if y is None:
        y = torch.empty((A.n,) if x.dim() == 1 else (A.n, k), dtype=torch.float32, device=x.device)
    _block(y, torch.float32, A.n, k, "y")
    _check(lib().pksell_spmv(ctypes.byref(A.desc), _ptr(x), _ptr(y), k, _stream(x.device)))
    return y


def spmv_static(A: PackSELLMatrix, x: torch.Tensor,
                y: torch.Tensor | None = None) -> torch.Tensor:
    """``spmv`` through pksell_spmv_static: products that need scratch take
    it from the library's per-GPU array, so the call allocates nothing
    (given y).  Concurrent calls on one GPU race on that array."""
    _block(x, torch.float32, A.m, None, "x")
    k = 1 if x.dim() == 1 else x.shape[1]
    if y is None:
        y = torch.empty((A.n,) if x.dim() == 1 else (A.n, k), dtype=torch.float32, device=x.device)
    _block(y, torch.float32, A.n, k, "y")
    _check(lib().pksell_spmv_static(ctypes.byref(A.desc), _ptr(x), _ptr(y), k,
                                    _stream(x.device)))
    return y


def spmv_f64(A: PackSELLMatrix, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """y = A_q x in float64 for a 64-bit-word (E11MY) matrix (x: m or m x k
    float64)."""
    _block(x, torch.float64, A.m, None, "x")
    k = 1 if x.dim() == 1 else x.shape[1]
    if y is None:
        y = torch.empty((A.n,) if x.dim() == 1 else (A.n, k), dtype=torch.float64, device=x.device)
    _block(y, torch.float64, A.n, k, "y")
    _check(lib().pksell_spmv_f64(ctypes.byref(A.desc), _ptr(x), _ptr(y), k, _stream(x.device)))
    return y


def spmv_t(A: PackSELLMatrix, g: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """y = A_q^T g (g: n or n x k float32)."""
    k = 1 if g.dim() == 1 else g.shape[1]
    _block(g, torch.float32, A.n, None, "g")
    if y is None:
        y = torch.empty((A.m,) if g.dim() == 1 else (A.m, k), dtype=torch.float32, device=g.device)
    _block(y, torch.float32, A.m, k, "y")
    _check(lib().pksell_spmv_t(ctypes.byref(A.desc), _ptr(g), _ptr(y), k, _stream(g.device)))
    return y


def grad_values(A: PackSELLMatrix, rowptr: torch.Tensor, g: torch.Tensor,
                x: torch.Tensor) -> torch.Tensor:
    """sum_s g[i, s] x[j, s] at every stored nonzero, in the CSR order of
    ``rowptr`` (g: n or n x k, x: m or m x k)."""
    k = 1 if g.dim() == 1 else g.shape[1]
    _block(g, torch.float32, A.n, None, "g")
    _block(x, torch.float32, A.m, k, "x")
    out = torch.empty(max(1, A.nnz), dtype=torch.float32, device=g.device)
    rp = _dev(rowptr, torch.int64, g.device)
    _check(lib().pksell_grad_values(ctypes.byref(A.desc), _ptr(rp), _ptr(g), _ptr(x),
                                    _ptr(out), k, _stream(g.device)))
    return out[:A.nnz]


def decode(A: PackSELLMatrix):
    """(column, value) at every word position (phantom rows left at 0)."""
    cols = torch.zeros(max(1, A.n_words), dtype=torch.int32, device=A.device)
    vals = torch.zeros(max(1, A.n_words), dtype=torch.float32, device=A.device)
    _check(lib().pksell_decode(ctypes.byref(A.desc), _ptr(cols), _ptr(vals), _stream(A.device)))
    return cols[:A.n_words], vals[:A.n_words]


class SellMatrix:
    """Plain SELL-C-sigma with float32, float64 or half values (the
    comparator); half-value matrices take float32 vectors."""

    def __init__(self, desc: CSell, tensors: dict, device):
        self.desc = desc
        self.t = tensors
        self.device = device

    n = property(lambda s: s.desc.n)
    m = property(lambda s: s.desc.m)
    n_slots = property(lambda s: s.desc.n_slots)

    @property
    def cache_hint(self) -> int:
        """CACHE_STREAM (the default) or CACHE_RESIDENT: how the C = 64
        float32-vector product loads the slots (same results either way)."""
        return self.desc.cache_hint

    @cache_hint.setter
    def cache_hint(self, v: int):
        self.desc.cache_hint = int(v)

    @property
    def dtype(self):
        """The vector (x, y) dtype."""
        return torch.float64 if self.desc.dtype == F64 else torch.float32

    @property
    def value_dtype(self):
        return {F64: torch.float64, F16: torch.float16}.get(self.desc.dtype, torch.float32)

    @property
    def paired(self) -> bool:
        """Column and value side by side in one 8-byte slot."""
        return self.desc.dtype == F32_PAIRED

    def bytes_per_spmv(self) -> int:
        d = self.desc
        vb = {F64: 8, F16: 2}.get(d.dtype, 4)  # value bytes per slot
        xb = 8 if d.dtype == F64 else 4        # vector element bytes
        b = (vb + 4) * d.n_slots + 8 * (d.n_slices + 1) + xb * (d.m + d.n)
        if d.perm_mode == IMPLICIT:
            b += d.perm_bytes * d.n
        return int(b)

    def replicate(self):
        t = {k: v.clone() for k, v in self.t.items()}
        desc = CSell.from_buffer_copy(self.desc)
        s = SellMatrix(desc, t, self.device)
        s._bind()
        return s

    def _bind(self):
        d = self.desc
        d.offset = self.t["offset"].data_ptr()
        d.perm = self.t["perm"].data_ptr() if self.t.get("perm") is not None else None
        d.col = self.t["col"].data_ptr() if self.t.get("col") is not None else None
        d.val = self.t["val"].data_ptr() if self.t.get("val") is not None else None


def sell_encode(rowptr, col, val, n: int, m: int, dtype=torch.float32, C: int = 64,
                sigma: int = 256, perm_mode: int = IMPLICIT, device="cuda",
                paired: bool = False) -> SellMatrix:
    """Plain SELL-C-sigma with ``dtype`` values (float32, float64 or half).
    ``paired`` (float32 only) stores each float32 value beside its int32
    column in one 8-byte slot, read with one load per slot."""
    device = torch.device(device)
    rp = _dev(rowptr, torch.int64, device)
    cl = _dev(col, torch.int32, device)
    vdt = torch.float64 if (isinstance(val, np.ndarray) and val.dtype == np.float64) or \
        (isinstance(val, torch.Tensor) and val.dtype == torch.float64) else torch.float32
    vl = _dev(val, vdt, device)
    code = {torch.float64: F64, torch.float16: F16}.get(dtype, F32)
    _require(not paired or code == F32, "paired slots hold float32 values")
    if paired:
        code = F32_PAIRED
    desc = CSell()
    ws_bytes = ctypes.c_size_t()
    L = lib()
    _check(L.pksell_sell_query(n, m, int(cl.numel()), C, sigma, code, perm_mode,
                               ctypes.byref(desc), ctypes.byref(ws_bytes)))
    t = {"offset": torch.empty(desc.n_slices + 1, dtype=torch.int64, device=device)}
    if perm_mode == IMPLICIT:
        t["perm"] = torch.empty(max(1, n * desc.perm_bytes), dtype=torch.uint8, device=device)
    ws = torch.empty(max(1, ws_bytes.value), dtype=torch.uint8, device=device)
    S = SellMatrix(desc, t, device)
    S._bind()
    st = _stream(device)
    vcode = F64 if vdt == torch.float64 else F32
    _check(L.pksell_sell_encode(_ptr(rp), _ptr(cl), _ptr(vl), vcode, ctypes.byref(desc),
                                _ptr(ws), ws_bytes.value, st))
    if paired:
        t["val"] = torch.empty(max(1, desc.n_slots), dtype=torch.int64, device=device)
    else:
        t["col"] = torch.empty(max(1, desc.n_slots), dtype=torch.int32, device=device)
        t["val"] = torch.empty(max(1, desc.n_slots), dtype=dtype, device=device)
    S._bind()
    _check(L.pksell_sell_encode(_ptr(rp), _ptr(cl), _ptr(vl), vcode, ctypes.byref(desc),
                                _ptr(ws), ws_bytes.value, st))
    return S


def sell_spmv(S: SellMatrix, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    if y is None:
        y = torch.empty(S.n, dtype=S.dtype, device=x.device)
    _block(x, S.dtype, S.m, 1, "x")
    _block(y, S.dtype, S.n, 1, "y")
    _check(lib().pksell_sell_spmv(ctypes.byref(S.desc), _ptr(x), _ptr(y), _stream(x.device)))
    return y


class Csr32Matrix:
    """Plain CSR with float32 values in 8-byte entries and a chunk plan (the
    comparator of the CSR-packed product)."""

    def __init__(self, desc: CCsr32, tensors: dict, device):
        self.desc = desc
        self.t = tensors
        self.device = device

    n = property(lambda s: s.desc.n)
    m = property(lambda s: s.desc.m)
    nnz = property(lambda s: s.desc.nnz)
    n_chunks = property(lambda s: s.desc.n_chunks)

    def bytes_per_spmv(self) -> int:
        d = self.desc
        return int(8 * d.nnz + 8 * (d.n + 1) + 4 * (d.n_chunks + 1) + 4 * d.m + 4 * d.n)

    def replicate(self):
        c = Csr32Matrix(CCsr32.from_buffer_copy(self.desc),
                        {k: v.clone() for k, v in self.t.items()}, self.device)
        c._bind()
        return c

    def _bind(self):
        d = self.desc
        d.rowptr = self.t["rowptr"].data_ptr()
        d.ent = self.t["ent"].data_ptr()
        d.lo = self.t["lo"].data_ptr()
        d.partial = self.t["partial"].data_ptr()


def csr32_encode(rowptr, col, val, n: int, m: int, T: int = 512, device="cuda") -> Csr32Matrix:
    """CSR (numpy or torch) -> float32 CSR entries with a chunk plan of T
    entries per chunk (256, 512 or 1024)."""
    device = torch.device(device)
    rp = _dev(rowptr, torch.int64, device)
    cl = _dev(col, torch.int32, device)
    f64 = (isinstance(val, np.ndarray) and val.dtype == np.float64) or \
        (isinstance(val, torch.Tensor) and val.dtype == torch.float64)
    vl = _dev(val, torch.float64 if f64 else torch.float32, device)
    nnz = int(cl.numel())
    _require(rp.numel() == n + 1, "rowptr must have n + 1 entries")
    desc = CCsr32()
    _check(lib().pksell_csr32_query(n, m, nnz, T, ctypes.byref(desc)))
    t = {"rowptr": rp,
         "ent": torch.empty(max(1, nnz), dtype=torch.int64, device=device),
         "lo": torch.empty(desc.n_chunks + 1, dtype=torch.int32, device=device),
         "partial": torch.empty(max(1, 3 * desc.n_chunks), dtype=torch.float32, device=device)}
    A = Csr32Matrix(desc, t, device)
    A._bind()
    _check(lib().pksell_csr32_encode(_ptr(cl), _ptr(vl), F64 if f64 else F32, ctypes.byref(desc),
                                     _stream(device)))
    return A


def csr32_spmv(A: Csr32Matrix, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """y = A x in float32 (x: m float32 on the device)."""
    _block(x, torch.float32, A.m, 1, "x")
    if y is None:
        y = torch.empty(A.n, dtype=torch.float32, device=x.device)
    _block(y, torch.float32, A.n, 1, "y")
    _check(lib().pksell_csr32_spmv(ctypes.byref(A.desc), _ptr(x), _ptr(y), _stream(x.device)))
    return y


class SolveInfo(dict):
    """Iteration counts, final true relative residual, wall seconds, status."""


def pcg(A_lo: PackSELLMatrix | None, A_hi, b: torch.Tensor,
        x0: torch.Tensor | None = None, tol: float = 1e-10, m_in: int = 50,
        max_outer: int = 10000, check: bool = True):
    """Solve A x = b: inner-outer CG with a PackSELL inner operator, or plain
    float64 CG when ``A_lo`` is None.  ``A_hi`` (the float64 operator) is a
    float64 SellMatrix or a 64-bit-word (E11MY) PackSELLMatrix.
    Returns (x, info)."""
    _block(b, torch.float64, A_hi.n, 1, "b")
    if x0 is not None:
        _block(x0, torch.float64, A_hi.n, 1, "x0")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    ws_bytes = ctypes.c_size_t()
    lo = ctypes.byref(A_lo.desc) if A_lo is not None else None
    L = lib()
    words64 = isinstance(A_hi, PackSELLMatrix)
    query = L.pksell_pcg64_workspace if words64 else L.pksell_pcg_workspace
    run = L.pksell_pcg64 if words64 else L.pksell_pcg
    _check(query(lo, ctypes.byref(A_hi.desc), ctypes.byref(ws_bytes)))
    ws = torch.empty(max(1, ws_bytes.value), dtype=torch.uint8, device=b.device)
    info = CPcgInfo()
    st = run(lo, ctypes.byref(A_hi.desc), _ptr(b), _ptr(x), tol, m_in, max_outer,
             ctypes.byref(info), _ptr(ws), ws_bytes.value, _stream(b.device))
    out = SolveInfo(outer_iterations=info.outer_iterations,
                    inner_iterations=info.inner_iterations,
                    rel_residual=info.rel_residual, seconds=info.seconds, status=st)
    if check and st not in (OK,):
        raise PackSELLError(st, L.pksell_last_error().decode())
    return x, out


def f3r(A1: "SellMatrix", b: torch.Tensor, A2: "SellMatrix | None" = None, A3=None,
        x0: torch.Tensor | None = None, tol: float = 1e-10, m1: int = 100, m2: int = 8,
        m3: int = 4, m4: int = 2, omega: float = 1.0, max_cycles: int = 100,
        check: bool = True):
    """Solve A x = b with the F3R nested solver (sec. 5.2.1).  ``A1`` is the
    float64 SELL operator of the outer layer.  With ``A2`` None every layer
    runs on A1 in float64 (FP64-F3R); otherwise ``A2`` (float32 SELL) is the
    second layer's operator and ``A3`` (half-value SELL, or a PackSELL matrix
    with 32-bit words) that of layers 3 and 4, with float32 vectors.
    Returns (x, info)."""
    _block(b, torch.float64, A1.n, 1, "b")
    _require(A2 is not None or A3 is None, "A3 needs A2 (the mixed-precision form)")
    _require(A2 is None or A3 is not None, "the mixed-precision form needs A3")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    _block(x, torch.float64, A1.n, 1, "x0")
    prm = CF3RParams(m1, m2, m3, m4, float(omega), max_cycles, 0)
    L = lib()
    ws_bytes = ctypes.c_size_t()
    _check(L.pksell_f3r_workspace(A1.n, int(A2 is not None), ctypes.byref(prm),
                                  ctypes.byref(ws_bytes)))
    ws = torch.empty(max(1, ws_bytes.value), dtype=torch.uint8, device=b.device)
    a2 = ctypes.byref(A2.desc) if A2 is not None else None
    a3s = ctypes.byref(A3.desc) if isinstance(A3, SellMatrix) else None
    a3p = ctypes.byref(A3.desc) if isinstance(A3, PackSELLMatrix) else None
    info = CPcgInfo()
    st = L.pksell_f3r(ctypes.byref(A1.desc), a2, a3s, a3p, _ptr(b), _ptr(x), tol,
                      ctypes.byref(prm), ctypes.byref(info), _ptr(ws), ws_bytes.value,
                      _stream(b.device))
    out = SolveInfo(outer_iterations=info.outer_iterations,
                    inner_iterations=info.inner_iterations,
                    rel_residual=info.rel_residual, seconds=info.seconds, status=st)
    if check and st != OK:
        raise PackSELLError(st, L.pksell_last_error().decode())
    return x, out


class BatchedSpMV:
    """Y_b = A_b X_b (or A_b^T G_b with ``transpose``) for a list of PackSELL
    matrices in one persistent launch; ``capture()`` records the launch in
    a HIP graph that ``replay()`` re-runs with the same buffers."""

    def __init__(self, mats: list, inputs: list, outputs: list, transpose: bool = False):
        _require(len(mats) == len(inputs) == len(outputs) and len(mats) > 0,
                 "mats, inputs and outputs must be non-empty lists of one length")
        self.mats, self.inputs, self.outputs = mats, inputs, outputs
        k = 1 if inputs[0].dim() == 1 else inputs[0].shape[1]
        dev = inputs[0].device
        arr = (CBatchItem * len(mats))()
        for i, (A, x, y) in enumerate(zip(mats, inputs, outputs)):
            rows_in, rows_out = (A.n, A.m) if transpose else (A.m, A.n)
            _block(x, torch.float32, rows_in, k, f"inputs[{i}]")
            _block(y, torch.float32, rows_out, k, f"outputs[{i}]")
            arr[i].A = ctypes.pointer(A.desc)
            arr[i].inp = x.data_ptr()
            arr[i].out = y.data_ptr()
        self._arr = arr
        nbytes = ctypes.c_size_t()
        L = lib()
        _check(L.pksell_batch_plan_bytes(len(mats), ctypes.byref(nbytes)))
        self.ws = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=dev)
        self.plan = CBatch()
        _check(L.pksell_batch_plan(arr, len(mats), k, 1 if transpose else 0,
                                   ctypes.byref(self.plan), _ptr(self.ws), nbytes.value,
                                   _stream(dev)))
        self.device = dev
        self.graph = None

    def __call__(self):
        _check(lib().pksell_spmv_batched(ctypes.byref(self.plan), _stream(self.device)))
        return self.outputs

    def capture(self):
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self()
        self.graph = g
        return self

    def replay(self):
        self.graph.replay()
        return self.outputs
