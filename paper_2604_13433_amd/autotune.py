"""Autotuner for PackSELL parameters: delta width D (the delta/value bit
split), slice height C, window sigma and, for single-vector products with
C = 64, the wide-slice split width J (the work-unit shape).

Model first, measurement second.  The encoder's analyse phase alone gives
the exact stored-word count (nonzeros + dummies + padding) of every
candidate, so the algorithmic bytes of one product are known without
building any words.  The product is bandwidth-bound, so the cheapest few
candidates by bytes are then encoded and timed on the GPU (HIP events over
graph replays), and the fastest wins.  The split width does not change the
bytes, only how the work is cut into waves, so each timed C = 64 candidate
is also timed with every J of ``split_list`` that splits at least one of its
slices.  For single-vector products the CSR-packed layout (C = 1, sigma = 1,
no padding, a product balanced over chunks of words) is a candidate too:
its fewest-bytes D is timed with every chunk size of ``csr_chunks``, and it
wins when it is faster.  Precision is a constraint, not a
goal: E8MY candidates keep at least ``min_mantissa`` mantissa bits
(Y = 22 - D), FIX at least ``min_mantissa`` value bits.

Results are cached in a JSON file keyed by a hash of the sparsity pattern
and the request.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import binding as B

DEFAULT_C = (32, 64)
DEFAULT_SIGMA = (64, 256, 1024, 8192, 65536)
DEFAULT_SPLIT = (128, 256)
DEFAULT_CSR_CHUNKS = (512,)


def signature(rowptr, col, n: int, m: int, fmt: str, min_mantissa: int, k: int) -> str:
    h = hashlib.blake2b(digest_size=16)
    h.update(np.asarray(rowptr, np.int64).tobytes())
    h.update(np.asarray(col, np.int32).tobytes())
    h.update(f"{n},{m},{fmt},{min_mantissa},{k}".encode())
    return h.hexdigest()


def d_candidates(fmt: str, min_mantissa: int):
    if fmt == "fp16":
        return [15]
    if fmt == "e8my":
        return list(range(1, 22 - min_mantissa + 1))
    if fmt == "fix":
        return list(range(1, 31 - min_mantissa + 1))
    raise ValueError(fmt)


def _time_spmv(A, x, y, reps=50):
    for _ in range(3):
        B.spmv(A, x, y)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(10):
            B.spmv(A, x, y)
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps // 10):
        g.replay()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / (reps // 10 * 10)


def tune(rowptr, col, val, n: int, m: int, fmt: str = "e8my", min_mantissa: int = 13,
         perm_mode: int = B.IMPLICIT, k: int = 1, C_list=DEFAULT_C, sigma_list=DEFAULT_SIGMA,
         split_list=DEFAULT_SPLIT, time_top: int = 3, cache_path: str | None = None,
         device="cuda", csr_chunks=DEFAULT_CSR_CHUNKS) -> dict:
    """Returns {"fmt", "D", "C", "sigma", "split_words", "bytes", "us",
    "candidates": [...], "csr_candidates": [...]}.  C = 1 and sigma = 1 with
    split_words > 0 selects the CSR-packed layout."""
    key = (signature(rowptr, col, n, m, fmt, min_mantissa, k) +
           f":{tuple(split_list)}:{tuple(csr_chunks)}")
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    device = torch.device(device)
    rp = torch.as_tensor(np.asarray(rowptr, np.int64)).to(device)
    cl = torch.as_tensor(np.asarray(col, np.int32)).to(device)
    vl = torch.as_tensor(np.asarray(val, np.float32)).to(device)
    cands = []
    for D in d_candidates(fmt, min_mantissa):
        for C in C_list:
            for sigma in sigma_list:
                if sigma < C:
                    continue
                A = B.encode(rp, cl, vl, n, m, fmt, D, C, sigma, perm_mode, device,
                             analyse_only=True)
                cands.append(dict(D=D, C=C, sigma=sigma, words=int(A.n_words),
                                  dummies=int(A.n_dummies), bytes=A.bytes_per_spmv(k)))
    cands.sort(key=lambda c: (c["bytes"], -c["C"], c["sigma"]))
    x = torch.rand((m,) if k == 1 else (m, k), device=device) * 2 - 1
    y = torch.empty((n,) if k == 1 else (n, k), device=device)
    for c in cands[:time_top]:
        A = B.encode(rp, cl, vl, n, m, fmt, c["D"], c["C"], c["sigma"], perm_mode, device)
        c["split_words"] = 0
        c["us"] = round(_time_spmv(A, x, y) * 1e3, 3)
        del A
        if k != 1 or c["C"] != 64:
            continue
        c["split_us"] = {}
        for J in split_list:
            A = B.encode(rp, cl, vl, n, m, fmt, c["D"], c["C"], c["sigma"], perm_mode, device,
                         split_words=J)
            if A.n_split_units > 0:
                c["split_us"][str(J)] = round(_time_spmv(A, x, y) * 1e3, 3)
            del A
        if c["split_us"]:
            J, us = min(c["split_us"].items(), key=lambda kv: kv[1])
            if us < c["us"]:
                c["split_words"], c["us"] = int(J), us
    timed = [c for c in cands if "us" in c]
    csr = []
    if k == 1 and csr_chunks:
        for D in d_candidates(fmt, min_mantissa):
            A = B.encode(rp, cl, vl, n, m, fmt, D, 1, 1, B.EXPLICIT, device,
                         analyse_only=True, split_words=int(csr_chunks[0]))
            csr.append(dict(D=D, C=1, sigma=1, words=int(A.n_words),
                            dummies=int(A.n_dummies), bytes=A.bytes_per_spmv(1)))
        csr.sort(key=lambda c: c["bytes"])
        c = csr[0]
        c["chunk_us"], chunk_bytes = {}, {}
        for T in csr_chunks:
            A = B.encode_packed_csr(rp, cl, vl, n, m, fmt, c["D"], int(T), device)
            c["chunk_us"][str(T)] = round(_time_spmv(A, x, y) * 1e3, 3)
            chunk_bytes[str(T)] = A.bytes_per_spmv(1)  # the plan's size depends on T
            del A
        T, us = min(c["chunk_us"].items(), key=lambda kv: kv[1])
        c["split_words"], c["us"], c["bytes"] = int(T), us, chunk_bytes[T]
        timed.append(c)
    best = min(timed, key=lambda c: c["us"])
    out = dict(fmt=fmt, D=best["D"], C=best["C"], sigma=best["sigma"],
               split_words=best["split_words"], bytes=best["bytes"], us=best["us"],
               min_mantissa=min_mantissa, k=k, candidates=cands[: max(10, time_top)],
               csr_candidates=csr[:5])
    if cache_path:
        cache[key] = out
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return out
