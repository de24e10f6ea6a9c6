"""PackSELL SpMV benchmark on one MI355X.

Workload: 3D 7-point variable-coefficient Laplacian on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760, lognormal(0, 0.5) edge coefficients),
x ~ U[-1, 1] float32.  One step = one PackSELL SpMV y = A_q x over the whole
matrix (FP16 values, D = 15, C = 64, sigma = 256, rows explicitly reordered
as in the paper's SpMV measurements).  The same product in E8M13 (D = 9)
PackSELL and in float32 / float64 SELL-C-sigma is timed the same way.

Timing: R replicas of every input (>= 1 GiB in total) rotate so the 256 MB
Infinity Cache cannot serve repeats from cache; the K timed launches are
replayed from HIP graphs (captured once, no host work between launches) and
bracketed by HIP events on the launch stream.  GB/s counts the algorithmic
bytes of one product (every stored word incl. padding and dummies, the
offsets, x once and y once).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# label -> (matrix, x, {variant: (y in original row order, fmt, D)}): products
# of the extra legs whose errors the CPU leg computes against the oracle
# (fmt None: only the eq. 5 backward error against the unquantised values)
EXTRA_CHECKS = {}


def record(label, mat, x, variant, y, fmt=None, D=0):
    """Keeps a product for the CPU leg's error check."""
    entry = EXTRA_CHECKS.setdefault(label, (mat, np.asarray(x), {}))
    entry[2][variant] = (np.asarray(y), fmt, D)


def sell_in_original_order(B, a, S, x):
    """A SELL comparator's product in the original row order: the same
    matrix encoded in implicit order (the same slots and sums per row; the
    explicit encoding keeps no perm to undo its sort)."""
    Si = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, S.value_dtype, S.desc.C, S.desc.sigma,
                       B.IMPLICIT, x.device, paired=S.paired)
    return B.sell_spmv(Si, x).cpu().numpy()


def original_order(B, A, y):
    """A product in stored row order (explicit mode) put back in the
    original row order with the matrix's perm."""
    y = y.cpu().numpy() if hasattr(y, "cpu") else np.asarray(y)
    if A.perm_mode == B.IMPLICIT or A.perm is None or A.sigma == 1:
        return y
    i = np.arange(A.n)
    orig = (i // A.sigma) * A.sigma + A.perm.cpu().numpy()[: A.n].astype(np.int64)
    out = np.empty_like(y)
    out[orig] = y
    return out
METRIC = "PackSELL SpMV GB/s and % HBM roofline vs FP32 SELL at stated err; PCG time-to-1e-10"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Hardware-counter HBM traffic of the headline kernel, from the committed
# rocprofv3 summary.  It is reported only while the kernel sources hash to
# the value recorded there (a changed kernel invalidates the counters).
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_spmv_pair_fp16_laplace3d_128.md")


def profiled_traffic(path=TRAFFIC_PROFILE):
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.split(":", 1)[0] in ("sources", "source_sha256",
                                                     "traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    for src in fields["sources"].split():
        try:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        except OSError:
            return None
    if h.hexdigest() != fields["source_sha256"]:
        log("[bench] headline kernel sources changed since the counters were taken: traffic null")
        return None
    return int(fields["traffic_bytes_per_launch"])


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=400)
    p.add_argument("--warmup", type=int, default=2000,
                   help="untimed launches first (about 30 ms of the headline product, so clocks settle)")
    p.add_argument("--grid", type=int, default=128, help="grid points per axis")
    p.add_argument("--replica-bytes", type=float, default=1.2e9)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--only", default="", help="comma list of variants to time")
    p.add_argument("--no-pcg", action="store_true", help="skip the solver leg")
    p.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the power-law and block-stencil legs")
    p.add_argument("--leg", default="", choices=["", "powerlaw", "trsv", "f3r", "pcg", "multirhs"],
                   help="run only this leg and print its JSON (for profiling one kernel)")
    p.add_argument("--calib-copy-mb", type=int, default=0,
                   help="first run one plain device copy of this many MiB (a known-size "
                        "kernel to scale hardware byte counters)")
    return p.parse_args()


class Timed:
    """Windows of exactly K launches of ``launch(i)`` replayed from HIP graphs
    on one stream; ``run`` returns the median window's ms per launch and
    keeps every window's figure in ``windows_ms``.  A graph holds as many
    whole rotations of the replicas as fit in one window (at most
    ``max_nodes`` launches): each replay leaves a gap of a few microseconds
    before its first kernel, which one rotation per graph (16 launches of
    the 128^3 product) spread as 0.37 us over every launch.  Each window is
    preceded by one untimed replay, so that its first launch is already
    queued when its start event is recorded.  Warm-up is at least
    ``warmup`` launches and at least ``min_warm_s`` of GPU work."""

    max_nodes = 1024
    min_warm_s = 0.025

    def __init__(self, torch, launch, n_rep: int, steps: int, warmup: int, windows: int = 5):
        self.torch = torch
        self.launch = launch
        self.n_rep = n_rep
        self.steps = steps
        self.warmup = warmup
        self.windows = windows
        self.windows_ms = []

    def _graph(self, count: int, start: int):
        torch = self.torch
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(count):
                self.launch((start + i) % self.n_rep)
        return g

    def run(self):
        torch = self.torch
        for i in range(min(self.warmup, 3)):  # eager warm-up, before capture
            self.launch(i % self.n_rep)
        torch.cuda.synchronize()
        # a window of K <= max_nodes launches is one graph of exactly K
        # launches (cycling through the replicas), else whole rotations
        if self.steps <= self.max_nodes:
            full = self.steps
        else:
            full = self.n_rep * max(1, self.max_nodes // self.n_rep)
        g_full = self._graph(full, 0)
        rem = self.steps % full
        g_rem = self._graph(rem, 0) if rem else None
        # warm-up: at least ``warmup`` launches and at least min_warm_s of
        # GPU work (an idle GPU runs its first launches slower)
        for _ in range(max(1, math.ceil(self.warmup / full))):
            g_full.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < self.min_warm_s:
            g_full.replay()
            torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        self.windows_ms = []
        for _ in range(self.windows):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            # one untimed replay ahead of the window keeps the GPU busy while
            # the host submits the timed replays, so the window does not
            # start with the host's submission latency
            g_full.replay()
            e0.record(st)
            for _ in range(self.steps // full):
                g_full.replay()
            if g_rem is not None:
                g_rem.replay()
            e1.record(st)
            e1.synchronize()
            torch.cuda.synchronize()
            self.windows_ms.append(e0.elapsed_time(e1) / self.steps)  # ms per launch
        return sorted(self.windows_ms)[len(self.windows_ms) // 2]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is described, not built)"}))
        sys.exit(2)
    import torch

    from paper_2604_13433_amd import binding as B
    from paper_2604_13433_amd import workloads as W

    dev = torch.device("cuda:0")
    B.lib()  # fail loudly if the library is missing
    if args.calib_copy_mb:
        nbytes = args.calib_copy_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst
    if args.leg:
        leg = {"powerlaw": powerlaw_leg, "trsv": trsv_leg, "f3r": f3r_leg,
               "pcg": pcg_leg, "multirhs": multirhs_only_leg}[args.leg]
        print(json.dumps({args.leg: leg(args, torch, B, W)}), flush=True)
        return
    g = args.grid
    t0 = time.time()
    a = W.m2_laplace3d(g)
    x_np = W.uniform_vector(a.m, 3)
    log(f"[bench] laplace3d {g}^3: n={a.n} nnz={a.nnz} generated in {time.time() - t0:.1f}s")

    variants = {}

    def add_packsell(name, fmt, D, mode):
        A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256, mode, dev)
        return name, A

    built = []
    only = set(filter(None, args.only.split(",")))
    specs = [("packsell_fp16", "fp16", 15, B.EXPLICIT),
             ("packsell_e8m13", "e8my", 9, B.EXPLICIT),
             ("packsell_fp16_implicit", "fp16", 15, B.IMPLICIT)]
    # the E8MY delta/value split: D = 1, 2 (FP32-level values, a dummy at
    # nearly every plane jump) and 12 beside the D = 9 above
    specs += [(f"packsell_e8m{22 - D}", "e8my", D, B.EXPLICIT) for D in (1, 2, 12)]
    for name, fmt, D, mode in specs:
        if only and name not in only:
            continue
        built.append(add_packsell(name, fmt, D, mode))
    if not only or "packed_csr_fp16" in only:
        # the same words row after row (no slices): what SELL's slicing buys on a stencil
        built.append(("packed_csr_fp16",
                      B.encode_packed_csr(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 512, dev)))
    sells = []
    for name, dt, paired in [("sell_fp32", torch.float32, False),
                             ("sell_fp32_paired", torch.float32, True),
                             ("sell_fp16", torch.float16, False),
                             ("sell_fp64", torch.float64, False)]:
        if only and name not in only:
            continue
        S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, dt, 64, 256, B.EXPLICIT, dev,
                          paired=paired)
        sells.append((name, S))
    torch.cuda.synchronize()

    x0 = torch.from_numpy(x_np).to(dev)
    results = {}
    for name, A in built:
        per = A.bytes_per_spmv()
        R = max(2, int(math.ceil(args.replica_bytes / per)))
        reps = [A] + [A.replicate() for _ in range(R - 1)]
        xs = [x0.clone() for _ in range(R)]
        ys = [torch.empty(a.n, dtype=torch.float32, device=dev) for _ in range(R)]
        tm = Timed(torch, lambda i: B.spmv(reps[i], xs[i], ys[i]), R, args.steps, args.warmup)
        ms = tm.run()
        gbs = per / (ms * 1e-3) / 1e9
        results[name] = dict(ms=ms, gbs=gbs, bytes=per, replicas=R, words=A.n_words,
                             dummies=A.n_dummies, gflops=2 * a.nnz / (ms * 1e-3) / 1e9,
                             y=ys[0], A=A, useful=per - 4 * (A.n_words - a.nnz),
                             windows_us=[round(w * 1e3, 3) for w in tm.windows_ms])
        log(f"[bench] {name}: {ms * 1e3:.2f} us  {gbs:.0f} GB/s  ({R} replicas, "
            f"{per / 1e6:.1f} MB/product)")
        del reps, xs
    for name, S in sells:
        per = S.bytes_per_spmv()
        R = max(2, int(math.ceil(args.replica_bytes / per)))
        reps = [S] + [S.replicate() for _ in range(R - 1)]
        xs = [x0.to(S.dtype).clone() for _ in range(R)]
        ys = [torch.empty(a.n, dtype=S.dtype, device=dev) for _ in range(R)]
        tm = Timed(torch, lambda i: B.sell_spmv(reps[i], xs[i], ys[i]), R, args.steps,
                   args.warmup)
        ms = tm.run()
        gbs = per / (ms * 1e-3) / 1e9
        vb = S.value_dtype.itemsize
        results[name] = dict(ms=ms, gbs=gbs, bytes=per, replicas=R, slots=S.n_slots,
                             gflops=2 * a.nnz / (ms * 1e-3) / 1e9, y=ys[0], S=S,
                             useful=per - (4 + vb) * (S.n_slots - a.nnz),
                             windows_us=[round(w * 1e3, 3) for w in tm.windows_ms])
        log(f"[bench] {name}: {ms * 1e3:.2f} us  {gbs:.0f} GB/s  ({R} replicas)")
        del reps, xs

    head = "packsell_fp16" if "packsell_fp16" in results else next(iter(results))
    H = results[head]
    ceiling = stream_ceiling(args, torch, B, H["bytes"])
    out = {
        "metric": METRIC,
        "value": round(H["gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms"],
        "timing": f"median of 5 windows of exactly {args.steps} launches each (graph replays "
                  f"bracketed by HIP events on the launch stream, each window preceded by "
                  f"one untimed replay); per-window figures in variants.*.windows_us",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"laplace3d_7pt_{g}^3 PackSELL {head} D={H['A'].D} C=64 "
                               f"sigma=256 explicit, one y=Ax per step",
                   "n": a.n, "nnz": a.nnz, "words": H["words"], "dummies": H["dummies"],
                   "bytes_per_step": H["bytes"], "replicas": H["replicas"]},
        "roofline": {"bound": "hbm", "achieved": round(H["gbs"], 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(H["gbs"] / PEAK_HBM_GBS, 4),
                     "traffic": profiled_traffic() if head == "packsell_fp16" else None},
        "stream_ceiling": {"GB/s": round(ceiling, 1), "bytes": H["bytes"] // 16 * 16,
                           "frac_of_ceiling": round(H["gbs"] / ceiling, 4),
                           "what": "one streaming-read launch of the headline's byte count"},
        "gflops": round(H["gflops"], 1),
        "variants": {},
    }
    base32 = results.get("sell_fp32")
    base16 = results.get("sell_fp16")
    # the fastest float32 product among the SELL forms
    fp32_ms = {k: results[k]["ms"] for k in ("sell_fp32", "sell_fp32_paired") if k in results}
    best32 = min(fp32_ms, key=fp32_ms.get) if fp32_ms else None
    out["best_fp32"] = best32
    for name, r in results.items():
        v = {"us": round(r["ms"] * 1e3, 2), "GB/s": round(r["gbs"], 1),
             "GFLOP/s": round(r["gflops"], 1), "hbm_frac": round(r["gbs"] / PEAK_HBM_GBS, 4),
             "bytes": r["bytes"], "replicas": r["replicas"],
             "useful_GB/s": round(r["useful"] / (r["ms"] * 1e-3) / 1e9, 1),
             "windows_us": r["windows_us"]}
        if base32 is not None:
            v["speedup_vs_sell_fp32"] = round(base32["ms"] / r["ms"], 3)
        if best32 is not None:
            v["speedup_vs_best_fp32"] = round(fp32_ms[best32] / r["ms"], 3)
        if base16 is not None and name.startswith("packsell_fp16"):
            # same values (binary16), 4 B per word against 6 B per SELL slot
            v["speedup_vs_sell_fp16"] = round(base16["ms"] / r["ms"], 3)
        out["variants"][name] = v

    def leg(key, fn, *fargs):
        # a leg that fails leaves its error in the line instead of ending the run
        try:
            out[key] = fn(*fargs)
        except Exception as e:  # noqa: BLE001
            import traceback
            traceback.print_exc()
            out[key] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.synchronize()

    if not args.no_adjoint and "packsell_fp16" in results:
        leg("adjoint", adjoint_leg, args, a, results["packsell_fp16"]["A"], torch, B, W)
        leg("multi_rhs", multirhs_leg, args, a, results["packsell_fp16"]["A"], torch, B, W)
    leg("encode_ms", encode_leg, a, torch, B)
    if not args.no_extra:
        leg("powerlaw", powerlaw_leg, args, torch, B, W)
        leg("block3_27pt", block_leg, args, torch, B, W)
        leg("laplace3d_256", large_leg, args, torch, B, W)
        leg("fp64_words", fp64_leg, args, a, torch, B, W)
        leg("words16", w16_leg, args, torch, B, W)
        leg("trsv", trsv_leg, args, torch, B, W)
    if not args.no_batched:
        leg("batched", batched_leg, args, torch, B, W)
    if not args.no_pcg:
        leg("pcg", pcg_leg, args, torch, B, W)
        leg("f3r", f3r_leg, args, torch, B, W)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_leg(args, a, x_np, results, H, torch)
    print(json.dumps(out), flush=True)


def stream_ceiling(args, torch, B, nbytes):
    """GB/s of the fastest streaming-read launch of ``nbytes`` (rounded down
    to 16) over a few load shapes, with the same replica rotation and graph
    replay as the products."""
    dev = torch.device("cuda:0")
    nb = nbytes // 16 * 16
    R = max(2, int(math.ceil(args.replica_bytes / nb)))
    bufs = [torch.ones(nb // 4, dtype=torch.float32, device=dev) for _ in range(R)]
    best = 0.0
    for width, chunks in ((4, 7), (4, 8), (4, 16), (16, 4), (16, 7), (16, 8)):
        rd = [B.StreamRead(b, width, chunks) for b in bufs]
        ms = Timed(torch, lambda i: rd[i](), R, args.steps, min(args.warmup, 400)).run()
        gbs = nb / (ms * 1e-3) / 1e9
        log(f"[bench] streaming read of {nb} B ({width} B x {chunks} chunks/wave): "
            f"{ms * 1e3:.2f} us {gbs:.0f} GB/s")
        best = max(best, gbs)
    del bufs
    return best


def adjoint_leg(args, a, A, torch, B, W):
    """grad_x = A^T g over the same words (atomic scatter) and the value
    gradient, on the same matrix and replica rotation as the forward."""
    dev = A.device
    per = A.bytes_per_spmv()
    R = max(2, int(math.ceil(args.replica_bytes / per)))
    reps = [A] + [A.replicate() for _ in range(R - 1)]
    gs = [torch.from_numpy(W.uniform_vector(a.n, 5)).to(dev) for _ in range(R)]
    outs = [torch.empty(a.m, dtype=torch.float32, device=dev) for _ in range(R)]
    ms = Timed(torch, lambda i: B.spmv_t(reps[i], gs[i], outs[i]), R, args.steps,
               args.warmup).run()
    # bytes: words + offsets + g once + the m outputs zeroed and accumulated
    bytes_t = 4 * A.n_words + 8 * (A.desc.n_slices + 1) + 4 * a.n + 8 * a.m
    log(f"[bench] spmv_t fp16: {ms * 1e3:.2f} us {bytes_t / (ms * 1e-3) / 1e9:.0f} GB/s")
    res = {"spmv_t_us": round(ms * 1e3, 2), "spmv_t_GB/s": round(bytes_t / (ms * 1e-3) / 1e9, 1)}
    del reps, outs
    # the same adjoint as a forward product on a PackSELL copy of (A_q)^T
    At = B.encode_transpose(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, dev)
    per_t = At.bytes_per_spmv()
    reps = [At] + [At.replicate() for _ in range(R - 1)]
    outs = [torch.empty(a.m, dtype=torch.float32, device=dev) for _ in range(R)]
    ms_t = Timed(torch, lambda i: B.spmv(reps[i], gs[i], outs[i]), R, args.steps,
                 args.warmup).run()
    log(f"[bench] adjoint via transposed copy: {ms_t * 1e3:.2f} us "
        f"{per_t / (ms_t * 1e-3) / 1e9:.0f} GB/s")
    res.update({"transposed_copy_us": round(ms_t * 1e3, 2),
                "transposed_copy_GB/s": round(per_t / (ms_t * 1e-3) / 1e9, 1),
                "speedup_vs_atomic": round(ms / ms_t, 2)})
    return res


def encode_leg(a, torch, B):
    """Wall time of the device encoder (analyse + fill) for the headline matrix."""
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(a.rowptr).to(dev)
    cl = torch.from_numpy(a.col).to(dev)
    vl = torch.from_numpy(a.val.astype(np.float32)).to(dev)
    B.encode(rp, cl, vl, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, dev)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(3):
        B.encode(rp, cl, vl, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, dev)
    torch.cuda.synchronize()
    return round((time.time() - t0) / 3 * 1e3, 2)


def time_variant(args, torch, B, A, m, n, mk_y=None):
    """ms per product for one PackSELL or SELL matrix with replica rotation."""
    dev = torch.device("cuda:0")
    per = A.bytes_per_spmv()
    R = max(2, int(math.ceil(args.replica_bytes / per)))
    reps = [A] + [A.replicate() for _ in range(R - 1)]
    if isinstance(A, B.SellMatrix):
        xs = [(torch.rand(m, device=dev, dtype=A.dtype) * 2 - 1) for _ in range(R)]
        ys = [torch.empty(n, dtype=A.dtype, device=dev) for _ in range(R)]
        fn = lambda i: B.sell_spmv(reps[i], xs[i], ys[i])
    else:
        xs = [(torch.rand(m, device=dev) * 2 - 1) for _ in range(R)]
        ys = [torch.empty(n, device=dev) for _ in range(R)]
        fn = lambda i: B.spmv(reps[i], xs[i], ys[i])
    ms = Timed(torch, fn, R, min(args.steps, 200), min(args.warmup, 20)).run()
    return ms, per, R


def time_csr32(args, torch, B, A):
    """ms per product of a float32 CSR comparator with replica rotation."""
    dev = torch.device("cuda:0")
    per = A.bytes_per_spmv()
    R = max(2, int(math.ceil(args.replica_bytes / per)))
    reps = [A] + [A.replicate() for _ in range(R - 1)]
    xs = [(torch.rand(A.m, device=dev) * 2 - 1) for _ in range(R)]
    ys = [torch.empty(A.n, device=dev) for _ in range(R)]
    ms = Timed(torch, lambda i: B.csr32_spmv(reps[i], xs[i], ys[i]), R, min(args.steps, 200),
               min(args.warmup, 20)).run()
    return ms, per, R


def powerlaw_leg(args, torch, B, W):
    """Irregular power-law rows, n = 10^6 (mean 30, max 5000, RSD 4.3):
    PackSELL FP16 and E8M10 (D = 12) at sigma = 65536 against FP32 SELL,
    with and without wide-slice splitting (J words per work unit), and the
    CSR-packed words (no padding, no sort) with the product balanced over
    chunks of J words."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    a = W.m3_powerlaw()
    log(f"[bench] powerlaw n={a.n} nnz={a.nnz} generated in {time.time() - t0:.1f}s")
    res = {"n": a.n, "nnz": a.nnz}
    variants = [("packsell_fp16", "fp16", 15, 0), ("packsell_e8m10", "e8my", 12, 0)]
    variants += [(f"packsell_fp16_split{J}", "fp16", 15, J) for J in (128, 256, 512)]
    variants += [("packsell_e8m10_split256", "e8my", 12, 256)]
    variants += [(f"packed_csr_fp16_chunk{J}", "fp16", 15, J) for J in (256, 512, 1024)]
    variants += [("packed_csr_e8m10_chunk512", "e8my", 12, 512)]
    # the E8MY delta/value split (D = 1, 2, 9; D = 12 above) and 16-bit fixed
    # point with a per-row scale (FIX, D = 15) on the best layout
    variants += [(f"packed_csr_e8m{22 - D}_chunk512", "e8my", D, 512) for D in (1, 2, 9)]
    variants += [("packed_csr_fix16_chunk512", "fix", 15, 512)]
    # --only (with --leg powerlaw) restricts the leg to the named variants
    only = set(filter(None, args.only.split(","))) if args.leg == "powerlaw" else set()
    want = lambda name: not only or name in only
    variants = [v for v in variants if want(v[0])]
    x_chk = torch.from_numpy(W.uniform_vector(a.m, 41)).to(dev)
    for name, fmt, D, J in variants:
        csr = name.startswith("packed_csr")
        if csr:
            A = B.encode_packed_csr(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, J, dev)
        else:
            A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 65536, B.EXPLICIT, dev,
                         split_words=J)
        ms, per, R = time_variant(args, torch, B, A, a.m, a.n)
        res[name] = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                     "GFLOP/s": round(2 * a.nnz / (ms * 1e-3) / 1e9, 1),
                     "words_per_nnz": round(A.n_words / a.nnz, 3)}
        if csr:
            res[name].update(chunk_words=J, chunks=A.n_units)
        else:
            res[name]["sigma"] = 65536
        if J and not csr:
            res[name].update(split_words=J, units=A.n_units, split_units=A.n_split_units)
        record("powerlaw", a, x_chk.cpu().numpy(), name, original_order(B, A, B.spmv(A, x_chk)),
               fmt, D)
        log(f"[bench] powerlaw {name}: {res[name]}")
        del A
    # four right-hand sides through the chunk product: one 16-byte gather per word
    if want("packed_csr_fp16_chunk512_k4"):
        A = B.encode_packed_csr(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 512, dev)
        per = A.bytes_per_spmv(4)
        R = max(2, int(math.ceil(args.replica_bytes / per)))
        reps = [A] + [A.replicate() for _ in range(R - 1)]
        xs = [torch.rand((a.m, 4), device=dev) * 2 - 1 for _ in range(R)]
        ys = [torch.empty((a.n, 4), device=dev) for _ in range(R)]
        ms = Timed(torch, lambda i: B.spmv(reps[i], xs[i], ys[i]), R, min(args.steps, 200),
                   min(args.warmup, 20)).run()
        res["packed_csr_fp16_chunk512_k4"] = {"us": round(ms * 1e3, 2),
                                              "us_per_rhs": round(ms * 1e3 / 4, 2),
                                              "GB/s": round(per / (ms * 1e-3) / 1e9, 1)}
        x4 = torch.from_numpy(W.uniform_vector(a.m, 42, k=4)).to(dev)
        y4 = B.spmv(A, x4).cpu().numpy()
        for c in (0, 3):
            record(f"powerlaw_k4_col{c}", a, x4[:, c].cpu().numpy(), "packed_csr_fp16_chunk512_k4",
                   y4[:, c], "fp16", 15)
        log(f"[bench] powerlaw packed_csr_fp16_chunk512_k4: {res['packed_csr_fp16_chunk512_k4']}")
        del reps, xs, ys, A
    if want("sell_fp32"):
        S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, 64, 65536, B.EXPLICIT, dev)
        ms, per, R = time_variant(args, torch, B, S, a.m, a.n)
        res["sell_fp32"] = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                            "slots_per_nnz": round(S.n_slots / a.nnz, 3)}
        record("powerlaw", a, x_chk.cpu().numpy(), "sell_fp32",
               sell_in_original_order(B, a, S, x_chk), "f32")
        log(f"[bench] powerlaw sell_fp32: {res['sell_fp32']}")
    if want("sell_fp32_paired"):
        S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, 64, 65536, B.EXPLICIT, dev,
                          paired=True)
        ms, per, R = time_variant(args, torch, B, S, a.m, a.n)
        res["sell_fp32_paired"] = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1)}
        record("powerlaw", a, x_chk.cpu().numpy(), "sell_fp32_paired",
               sell_in_original_order(B, a, S, x_chk), "f32")
        log(f"[bench] powerlaw sell_fp32_paired: {res['sell_fp32_paired']}")
        del S
    # float32 CSR balanced over entry chunks (the CSR-packed product's own
    # scheme with plain 8-byte entries): the like-for-like float32 form here
    for T in (256, 512, 1024):
        if not want(f"csr32_chunk{T}"):
            continue
        Cm = B.csr32_encode(a.rowptr, a.col, a.val, a.n, a.m, T, dev)
        ms, per, R = time_csr32(args, torch, B, Cm)
        res[f"csr32_chunk{T}"] = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                                  "chunks": Cm.n_chunks}
        record("powerlaw", a, x_chk.cpu().numpy(), f"csr32_chunk{T}",
               B.csr32_spmv(Cm, x_chk).cpu().numpy(), "f32")
        log(f"[bench] powerlaw csr32_chunk{T}: {res[f'csr32_chunk{T}']}")
        del Cm
    fp32 = [k for k in ("sell_fp32", "sell_fp32_paired", "csr32_chunk256", "csr32_chunk512",
                        "csr32_chunk1024") if k in res]
    if fp32:
        best = min(fp32, key=lambda k: res[k]["us"])
        res["best_fp32"] = best
        for name, *_ in variants:
            if "sell_fp32" in res:
                res[name]["speedup_vs_sell_fp32"] = round(res["sell_fp32"]["us"] / res[name]["us"], 3)
            res[name]["speedup_vs_best_fp32"] = round(res[best]["us"] / res[name]["us"], 3)
    return res


def trsv_leg(args, torch, B, W):
    """Lower-triangular solve, level by level, on the lower triangle of the
    7-point 128^3 variable-coefficient Laplacian (lognormal(0, 0.5) edge
    coefficients; 382 levels):
    CSR-packed FP16 words against plain CSR with float32 values."""
    import copy
    import scipy.sparse as sp
    dev = torch.device("cuda:0")
    a = W.m2_laplace3d(args.grid)
    L = sp.tril(sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m))).tocsr()
    L.sort_indices()
    rp, cl, vl = L.indptr.astype(np.int64), L.indices.astype(np.int32), L.data
    res = {"n": a.n, "nnz": int(L.nnz)}
    b = torch.from_numpy(W.uniform_vector(a.n, 8)).to(dev)
    for name, fmt in (("packed_fp16", "fp16"), ("csr_fp32", None)):
        S = B.TriangularSolve(rp, cl, vl, a.n, fmt, 15, dev)
        per = S.bytes_per_solve()
        R = max(2, int(math.ceil(args.replica_bytes / per)))
        reps = [S]
        for _ in range(R - 1):
            c = copy.copy(S)
            if fmt is None:
                c.rp, c.cl, c.val = S.rp.clone(), S.cl.clone(), S.val.clone()
            else:
                c.L = S.L.replicate()
            reps.append(c)
        ys = [torch.empty(a.n, device=dev) for _ in range(R)]
        ms = Timed(torch, lambda i: reps[i](b, ys[i]), R, min(args.steps, 40),
                   min(args.warmup, 20)).run()
        res[name] = {"us": round(ms * 1e3, 1), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                     "levels": S.n_levels, "bytes": per,
                     "us_per_level": round(ms * 1e3 / S.n_levels, 2)}
        log(f"[bench] trsv {name}: {res[name]}")
        del reps, ys
    res["speedup_vs_csr_fp32"] = round(res["csr_fp32"]["us"] / res["packed_fp16"]["us"], 3)
    return res


def fp64_leg(args, a, torch, B, W):
    """64-bit-word PackSELL (E11MY, 8 bytes per stored word) against FP64
    SELL (12 bytes per slot), float64 x and y, on the 7-point 128^3
    Laplacian (D = 15: E11M36, no dummies) and on the scaled 27-point 100^3
    system of the solver leg (D = 14: E11M37), with the largest relative
    change of the product against the unquantised float64 matrix."""
    dev = torch.device("cuda:0")
    res = {}
    for name, mat, D, mode in [("laplace3d_128", a, 15, B.EXPLICIT),
                               ("stencil27_100", W.symmetric_diag_scale(W.m4_stencil27()), 14,
                                B.IMPLICIT)]:
        A = B.encode(mat.rowptr, mat.col, mat.val, mat.n, mat.m, "e11my", D, 64, 256, mode, dev)
        S = B.sell_encode(mat.rowptr, mat.col, mat.val, mat.n, mat.m, torch.float64, 64, 256, mode,
                          dev)
        per_p, per_s = A.bytes_per_spmv(), S.bytes_per_spmv()
        out = {}
        for label, M, per, fn in [("packsell64", A, per_p, B.spmv_f64), ("sell_fp64", S, per_s,
                                                                         B.sell_spmv)]:
            R = max(2, int(math.ceil(args.replica_bytes / per)))
            reps = [M] + [M.replicate() for _ in range(R - 1)]
            xs = [torch.rand(mat.m, dtype=torch.float64, device=dev) * 2 - 1 for _ in range(R)]
            ys = [torch.empty(mat.n, dtype=torch.float64, device=dev) for _ in range(R)]
            ms = Timed(torch, lambda i: fn(reps[i], xs[i], ys[i]), R, min(args.steps, 200),
                       min(args.warmup, 400)).run()
            out[label] = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                          "bytes": per}
            if label == "packsell64":
                yp = ys[0].clone()
                x0 = xs[0]
                record(f"fp64_words_{name}", mat, x0.cpu().numpy(), "packsell64",
                       original_order(B, M, fn(M, x0)), "e11my", D)
            else:
                ys_ref = fn(M, x0)  # same x, unquantised FP64 values
                record(f"fp64_words_{name}", mat, x0.cpu().numpy(), "sell_fp64",
                       sell_in_original_order(B, mat, M, x0), "f64")
            del reps, xs, ys
        diff = float((yp - ys_ref).abs().max() / ys_ref.abs().max().clamp_min(1e-300))
        out["speedup_vs_sell_fp64"] = round(out["sell_fp64"]["us"] / out["packsell64"]["us"], 3)
        out["D"] = D
        out["words"] = A.n_words
        out["max_rel_change_vs_fp64_values"] = diff
        res[name] = out
        log(f"[bench] 64-bit words {name}: {out}")
        del A, S
    return res


def large_leg(args, torch, B, W):
    """Extra (not one of the benchmark configs): the same 7-point Laplacian on
    a 256^3 grid (n = 16.8 M, about 600 MB per FP16 product), where the fixed
    start-up and tail of a launch weigh 8 times less than at 128^3: PackSELL
    FP16 and FP32 SELL against a streaming read of the same byte count."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    a = W.m2_laplace3d(256)
    log(f"[bench] laplace3d 256^3: n={a.n} nnz={a.nnz} generated in {time.time() - t0:.1f}s")
    res = {"n": a.n, "nnz": a.nnz}
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, dev)
    ms, per, R = time_variant(args, torch, B, A, a.m, a.n)
    res["packsell_fp16"] = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                            "hbm_frac": round(per / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                            "bytes": per}
    del A
    S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, 64, 256, B.EXPLICIT, dev)
    ms_s, per_s, _ = time_variant(args, torch, B, S, a.m, a.n)
    res["sell_fp32"] = {"us": round(ms_s * 1e3, 2), "GB/s": round(per_s / (ms_s * 1e-3) / 1e9, 1)}
    res["speedup_vs_sell_fp32"] = round(ms_s / ms, 3)
    del S
    ceil = stream_ceiling(args, torch, B, per)
    res["stream_ceiling_GB/s"] = round(ceil, 1)
    res["frac_of_ceiling"] = round(res["packsell_fp16"]["GB/s"] / ceil, 4)
    log(f"[bench] laplace3d 256^3: {res}")
    return res


def block_leg(args, torch, B, W):
    """Extra (not one of the benchmark configs): a 3-unknown 27-point block
    stencil on a 48^3 grid (81 nonzeros per row in runs of 9), where a tiny
    delta field suffices -- PackSELL E8M20 (D = 2) against FP32 SELL, with
    the backward error (eq. 5) of both against the float64 product."""
    dev = torch.device("cuda:0")
    a = W.block_stencil((48, 48, 48), 3, 8)
    x = torch.from_numpy(W.uniform_vector(a.m, 9)).to(dev)
    res = {"n": a.n, "nnz": a.nnz}
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", 2, 64, 256, B.IMPLICIT, dev)
    S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, 64, 256, B.IMPLICIT, dev)
    ms_p, per_p, _ = time_variant(args, torch, B, A, a.m, a.n)
    ms_s, per_s, _ = time_variant(args, torch, B, S, a.m, a.n)
    res["packsell_e8m20"] = {"us": round(ms_p * 1e3, 2), "GB/s": round(per_p / (ms_p * 1e-3) / 1e9, 1),
                             "words": A.n_words, "dummies": A.n_dummies}
    res["sell_fp32"] = {"us": round(ms_s * 1e3, 2), "GB/s": round(per_s / (ms_s * 1e-3) / 1e9, 1)}
    res["speedup_vs_sell_fp32"] = round(ms_s / ms_p, 3)
    Sp = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, 64, 256, B.IMPLICIT, dev,
                       paired=True)
    ms_q, per_q, _ = time_variant(args, torch, B, Sp, a.m, a.n)
    res["sell_fp32_paired"] = {"us": round(ms_q * 1e3, 2),
                               "GB/s": round(per_q / (ms_q * 1e-3) / 1e9, 1)}
    res["speedup_vs_best_fp32"] = round(min(ms_s, ms_q) / ms_p, 3)
    # errors against the float64 oracle are computed in the CPU leg
    x_np = x.cpu().numpy()
    record("block3_27pt", a, x_np, "packsell_e8m20", B.spmv(A, x).cpu().numpy(), "e8my", 2)
    record("block3_27pt", a, x_np, "sell_fp32", B.sell_spmv(S, x).cpu().numpy(), "f32")
    record("block3_27pt", a, x_np, "sell_fp32_paired", B.sell_spmv(Sp, x).cpu().numpy(), "f32")
    log(f"[bench] block3_27pt: {res}")
    return res


def w16_leg(args, torch, B, W):
    """16-bit words against 32-bit words and half-value SELL on the same
    matrix, explicit order, sigma = 256: E5M2 values (E5MY, D = 7) on the
    7-point 128^3 Laplacian, and 4-bit FIX16 (D = 11, exact for the 4 / -1
    values) on the 5-point 2048^2 Poisson matrix.  Backward errors (eq. 5)
    against the float64 product are computed in the CPU leg."""
    dev = torch.device("cuda:0")
    out = {}
    for label, a, fmt, D in (("laplace3d_128_e5m2", W.m2_laplace3d(128), "e5my", 7),
                             ("poisson2d_2048_fix16_int4", W.poisson2d(2048), "fix16", 11)):
        res = {"n": a.n, "nnz": a.nnz}
        x = torch.from_numpy(W.uniform_vector(a.m, 13)).to(dev)
        for name, mk in ((f"packsell16_{fmt}", lambda: B.encode(a.rowptr, a.col, a.val, a.n, a.m,
                                                                  fmt, D, 64, 256, B.EXPLICIT,
                                                                  dev)),
                         ("packsell_fp16", lambda: B.encode(a.rowptr, a.col, a.val, a.n, a.m,
                                                            "fp16", 15, 64, 256, B.EXPLICIT,
                                                            dev)),
                         ("sell_fp16", lambda: B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m,
                                                             torch.float16, 64, 256, B.EXPLICIT,
                                                             dev))):
            M = mk()
            ms, per, _ = time_variant(args, torch, B, M, a.m, a.n)
            r = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                 "hbm_frac": round(per / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4), "bytes": per}
            if isinstance(M, B.PackSELLMatrix):
                r["words"], r["dummies"] = M.n_words, M.n_dummies
                # product in the original row order for the error check
                record(label, a, x.cpu().numpy(), name, original_order(B, M, B.spmv(M, x)),
                       fmt if name.startswith("packsell16") else "fp16",
                       D if name.startswith("packsell16") else 15)
            res[name] = r
            del M
        for name in list(res):
            if name.startswith("packsell16"):
                res["speedup_vs_packsell_fp16"] = round(res["packsell_fp16"]["us"] / res[name]["us"], 3)
                res["speedup_vs_sell_fp16"] = round(res["sell_fp16"]["us"] / res[name]["us"], 3)
        log(f"[bench] 16-bit words {label}: {res}")
        out[label] = res
    return out


def multirhs_leg(args, a, A, torch, B, W):
    """Y = A_q X on the headline matrix for k = 8 and 32 right-hand sides
    (row-major blocks; lane groups of 2 and 8 lanes per row)."""
    dev = A.device
    res = {}
    for k in (8, 32):
        per = A.bytes_per_spmv(k)
        R = max(2, int(math.ceil(args.replica_bytes / per)))
        reps = [A] + [A.replicate() for _ in range(R - 1)]
        xs = [torch.from_numpy(W.uniform_vector(a.m, 20 + i, k=k)).to(dev) for i in range(R)]
        ys = [torch.empty((a.n, k), device=dev) for _ in range(R)]
        steps = max(R, min(args.steps, 100) // R * R)
        ms = Timed(torch, lambda i: B.spmv(reps[i], xs[i], ys[i]), R, steps,
                   min(args.warmup, 10)).run()
        res[f"k{k}"] = {"us": round(ms * 1e3, 2), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                        "GFLOP/s": round(2 * a.nnz * k / (ms * 1e-3) / 1e9, 1), "bytes": per,
                        "replicas": R}
        yk = original_order(B, A, B.spmv(A, xs[0]))
        for c in (0, k - 1):
            record(f"multi_rhs_k{k}_col{c}", a, xs[0][:, c].cpu().numpy(), "packsell_fp16",
                   yk[:, c], "fp16", 15)
        log(f"[bench] single-matrix k={k}: {res[f'k{k}']}")
        del reps, xs, ys
    return res


def multirhs_only_leg(args, torch, B, W):
    """The multi-RHS leg by itself, on the headline matrix (for profiling)."""
    a = W.m2_laplace3d(args.grid)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT,
                 torch.device("cuda:0"))
    return multirhs_leg(args, a, A, torch, B, W)


def batched_leg(args, torch, B, W):
    """64 stencils (n log-uniform in [1e4, 5e5]), E8M13, k = 1, 8, 32: one
    persistent launch over all matrices per step, replayed from a graph."""
    dev = torch.device("cuda:0")
    mats = W.m5_batch()
    enc = [B.encode(m.rowptr, m.col, m.val, m.n, m.m, "e8my", 9, 64, 256, B.IMPLICIT, dev)
           for m in mats]
    nnz = sum(m.nnz for m in mats)
    res = {"matrices": len(mats), "rows": sum(m.n for m in mats), "nnz": nnz,
           "words": sum(A.n_words for A in enc)}
    for k in (1, 8, 32):
        per = sum(A.bytes_per_spmv(k) for A in enc)
        R = max(1, min(4, int(math.ceil(args.replica_bytes / per))))
        sets = [enc] + [[A.replicate() for A in enc] for _ in range(R - 1)]
        bats = []
        for r in range(R):
            xs = [torch.from_numpy(W.uniform_vector(m.m, i, k=k)).to(dev) for i, m in enumerate(mats)]
            ys = [torch.empty((m.n,) if k == 1 else (m.n, k), device=dev) for m in mats]
            bats.append(B.BatchedSpMV(sets[r], xs, ys))
        steps = max(R, min(args.steps, 100) // R * R)
        ms = Timed(torch, lambda i: bats[i](), R, steps, min(args.warmup, 10)).run()
        res[f"k{k}"] = {"us": round(ms * 1e3, 1), "GB/s": round(per / (ms * 1e-3) / 1e9, 1),
                        "GFLOP/s": round(2 * nnz * k / (ms * 1e-3) / 1e9, 1),
                        "bytes": per, "replicas": R}
        bats[0]()
        torch.cuda.synchronize()
        for i in (0, len(mats) // 2, len(mats) - 1):  # implicit order: original rows
            xi, yi = bats[0].inputs[i].cpu().numpy(), bats[0].outputs[i].cpu().numpy()
            c = k - 1
            record(f"batched_k{k}_m{i}", mats[i], xi if k == 1 else xi[:, c], "packsell_e8m13",
                   yi if k == 1 else yi[:, c], "e8my", 9)
        log(f"[bench] batched k={k}: {ms * 1e3:.1f} us {per / (ms * 1e-3) / 1e9:.0f} GB/s")
        del bats, sets
    return res


def pcg_leg(args, torch, B, W):
    """Time to a 1e-10 relative residual on the SPD 27-point 100^3 stencil
    (lognormal(0, 1) edges, symmetrically scaled, b = A 1, x0 = 0): float64
    CG against the inner-outer CG with PackSELL E8MY inner products."""
    dev = torch.device("cuda:0")
    a = W.symmetric_diag_scale(W.m4_stencil27())
    b = torch.from_numpy(W.ones_rhs(a)).to(dev)
    hi = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float64, 64, 256, B.IMPLICIT, dev)
    res = {"workload": "stencil27 100^3 lognormal(0,1), Gbar^-1 A Gbar^-1, b = A 1, tol 1e-10",
           "n": a.n, "nnz": a.nnz}

    def run(lo, m_in, reps=3):
        times, info = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            x, info = B.pcg(lo, hi, b, tol=1e-10, m_in=m_in, max_outer=20000)
            times.append(info["seconds"])
        err = float((x - 1.0).abs().max())
        return dict(ms=round(1e3 * sorted(times)[len(times) // 2], 2),
                    iterations=info["outer_iterations"], inner=info["inner_iterations"],
                    rel_residual=info["rel_residual"], max_abs_err_vs_ones=err)

    res["fp64_cg"] = run(None, 0)
    log(f"[bench] fp64 CG: {res['fp64_cg']}")
    best = None
    for D in (9, 12, 14):
        lo = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", D, 64, 256, B.IMPLICIT, dev)
        for m_in in (20, 50, 80):
            r = run(lo, m_in)
            r["speedup_vs_fp64_cg"] = round(res["fp64_cg"]["ms"] / r["ms"], 3)
            res[f"iocg_e8m{22 - D}_min{m_in}"] = r
            log(f"[bench] IO-CG E8M{22 - D} m_in={m_in}: {r}")
            if best is None or r["ms"] < best[1]["ms"]:
                best = (f"iocg_e8m{22 - D}_min{m_in}", r)
    res["best"] = best[0]
    res["best_speedup_vs_fp64_cg"] = best[1]["speedup_vs_fp64_cg"]
    # the float64 operator as 64-bit-word PackSELL (E11M37, D = 14): it holds
    # A rounded to 38 significant bits, so these solve that system; the
    # FP64 SELL CG above stays the baseline of every speedup
    hi64 = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e11my", 14, 64, 256, B.IMPLICIT, dev)
    res["fp64_cg_words64"] = run_with(hi64, None, 0, run_fn=B.pcg, b=b)
    log(f"[bench] FP64 CG, 64-bit-word operator: {res['fp64_cg_words64']}")
    lo = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", 14, 64, 256, B.IMPLICIT, dev)
    r = run_with(hi64, lo, 20, run_fn=B.pcg, b=b)
    r["speedup_vs_fp64_cg"] = round(res["fp64_cg"]["ms"] / r["ms"], 3)
    res["iocg_e8m8_min20_words64_outer"] = r
    log(f"[bench] IO-CG E8M8 m_in=20, 64-bit-word outer: {r}")
    # 16-bit-word inner operators: fewer bytes, coarser values, more restarts
    for fmt, D, label in (("e5my", 4, "iocg_w16_e5m5_min20"), ("fix16", 7, "iocg_w16_int8_min20")):
        lo16 = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256, B.IMPLICIT, dev)
        r = run_with(hi, lo16, 20, run_fn=B.pcg, b=b)
        r["speedup_vs_fp64_cg"] = round(res["fp64_cg"]["ms"] / r["ms"], 3)
        r["words_per_row"] = round(lo16.n_words / a.n, 2)
        res[label] = r
        log(f"[bench] IO-CG {label}: {r}")
        del lo16
    return res


def f3r_leg(args, torch, B, W):
    """Time to a 1e-10 relative residual with the F3R nested solver (sec.
    5.2.1; outer FGMRES(100), FGMRES(8), FGMRES(4), Richardson(2)) in its
    three forms: every layer float64 (FP64-F3R); float32 SELL (paired
    8-byte slots) in layer 2 and half-value SELL in layers 3-4 (FP16-F3R);
    the same with FP16 PackSELL words in layers 3-4 (PackSELL-F3R).  On the SPD 27-point 100^3 system
    (b = A 1) and a nonsymmetric 7-point convection-diffusion 128^3 system
    (b ~ U[0, 1)), both symmetrically scaled."""
    dev = torch.device("cuda:0")
    out = {}
    for label, a, bvec in (
            ("stencil27_100", W.symmetric_diag_scale(W.m4_stencil27()), None),
            ("convdiff7_128", W.symmetric_diag_scale(W.convdiff3d(128, 11)), "uniform")):
        b_np = W.ones_rhs(a) if bvec is None else np.random.default_rng(12).uniform(0, 1, a.n)
        b = torch.from_numpy(b_np).to(dev)
        enc = lambda dt, paired=False: B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, dt, 64, 256,
                                                     B.IMPLICIT, dev, paired=paired)
        # layer 2: float32 SELL with paired 8-byte slots (the faster float32 form)
        A1, A2, A3s = enc(torch.float64), enc(torch.float32, True), enc(torch.float16)
        A3p = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.IMPLICIT, dev)
        res = {"n": a.n, "nnz": a.nnz, "params": "m1=100 m2=8 m3=4 m4=2 omega=1"}
        xs = {}
        # the *_resident forms set cache_hint RESIDENT on the layer 3-4 operator
        # (applied 64 times per outer step), so that it can stay in the
        # last-level cache between its products
        A3s_r, A3p_r = A3s.replicate(), A3p.replicate()
        A3s_r.cache_hint = A3p_r.cache_hint = B.CACHE_RESIDENT
        for name, kw in (("fp64_f3r", {}), ("fp16_f3r", dict(A2=A2, A3=A3s)),
                         ("packsell_f3r", dict(A2=A2, A3=A3p)),
                         ("fp16_f3r_resident", dict(A2=A2, A3=A3s_r)),
                         ("packsell_f3r_resident", dict(A2=A2, A3=A3p_r))):
            times, info, x = [], None, None
            for _ in range(5):
                x, info = B.f3r(A1, b, tol=1e-10, **kw)
                times.append(info["seconds"])
            xs[name] = x
            true = float(np.linalg.norm(b_np - csr_apply(a, x.cpu().numpy())) /
                         np.linalg.norm(b_np))
            res[name] = dict(ms=round(1e3 * sorted(times)[2], 2),
                             ms_all=[round(1e3 * t, 2) for t in times],
                             outer_steps=info["outer_iterations"], rel_residual=info["rel_residual"],
                             true_rel_residual_host=true)
            log(f"[bench] F3R {label} {name}: {res[name]}")
        for name in ("fp16_f3r", "packsell_f3r", "fp16_f3r_resident", "packsell_f3r_resident"):
            res[name]["speedup_vs_fp64_f3r"] = round(res["fp64_f3r"]["ms"] / res[name]["ms"], 3)
        res["packsell_over_fp16_speedup"] = round(res["fp16_f3r"]["ms"] / res["packsell_f3r"]["ms"], 3)
        res["packsell_over_fp16_speedup_resident"] = round(
            res["fp16_f3r_resident"]["ms"] / res["packsell_f3r_resident"]["ms"], 3)
        res["fp16_and_packsell_iterates_identical"] = bool(
            torch.equal(xs["fp16_f3r"], xs["packsell_f3r"]) and
            torch.equal(xs["fp16_f3r"], xs["fp16_f3r_resident"]) and
            torch.equal(xs["packsell_f3r"], xs["packsell_f3r_resident"]))
        out[label] = res
        del A1, A2, A3s, A3p, A3s_r, A3p_r
    return out


def csr_apply(a, x):
    """A x in float64 on the host with scipy (a residual check, not timed)."""
    import scipy.sparse as sp
    return sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m)) @ x


def run_with(hi, lo, m_in, run_fn, b, reps=3):
    """Median time of ``reps`` solves to 1e-10 (x0 = 0)."""
    times, info, x = [], None, None
    for _ in range(reps):
        x, info = run_fn(lo, hi, b, tol=1e-10, m_in=max(m_in, 1), max_outer=20000)
        times.append(info["seconds"])
    return dict(ms=round(1e3 * sorted(times)[len(times) // 2], 2),
                iterations=info["outer_iterations"], inner=info["inner_iterations"],
                rel_residual=info["rel_residual"],
                max_abs_err_vs_ones=float((x - 1.0).abs().max()))


def quantised(m, fmt, D):
    """The oracle's values of the matrix as a product of format ``fmt``
    holds them (None: no format, only the backward error is reported)."""
    from oracle import formats as F
    from oracle import packsell as P
    from oracle import packsell16 as P16
    from oracle import packsell64 as P64

    if fmt is None:
        return None
    if fmt == "f32":
        return m.val.astype(np.float32).astype(np.float64)
    if fmt == "f64":
        return m.val
    if fmt == "e11my":
        return P64.quantized(m.val, D)
    if fmt in ("e5my", "fix16"):
        return P16.quantized(m.rowptr, m.val, m.n, {"e5my": P16.FMT_E5MY,
                                                    "fix16": P16.FMT_FIX16}[fmt], D)
    code = {"fp16": F.FMT_FP16, "e8my": F.FMT_E8MY, "fix": F.FMT_FIX}[fmt]
    return P.quantized_values(m.rowptr, m.col, m.val, m.n, code, D)


def cpu_leg(args, a, x_np, results, H, torch):
    """The float64 CSR oracle timed on the host cores (and the error of every
    GPU result against it, which needs the oracle anyway)."""
    from oracle import formats as F
    from oracle import linalg as L
    from oracle import native
    from oracle import packsell as P

    q16 = P.quantized_values(a.rowptr, a.col, a.val, a.n, F.FMT_FP16, 15)
    # the oracle's own bytes: float64 CSR (8 B value + 4 B column per entry,
    # the int64 row pointer, float64 x and y once)
    csr_bytes = 12 * a.nnz + 8 * (a.n + 1) + 8 * a.m + 8 * a.n

    def timed(seconds):
        reps, t0 = 0, time.time()
        while True:
            L.spmv(a.rowptr, a.col, q16, x_np)
            reps += 1
            if time.time() - t0 >= seconds:
                return (time.time() - t0) / reps, reps

    cores = native.num_threads()
    dt, reps = timed(args.cpu_seconds / 2)
    native.set_num_threads(1)
    dt1, reps1 = timed(args.cpu_seconds / 2)
    native.set_num_threads(cores)
    errors = {}
    for name, r in results.items():
        y = r["y"].double().cpu().numpy()
        if name.startswith("packsell"):
            A = r["A"]
            fmt = F.FMT_FP16 if A.fmt == 0 else F.FMT_E8MY
            q = P.quantized_values(a.rowptr, a.col, a.val, a.n, fmt, A.D)
            E = P.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, A.D, 64, 256, A.perm_mode)
            ref = L.spmv(a.rowptr, a.col, q, x_np)
            if A.perm_mode == 0:
                ref = ref[E.stored_rows]
                full = L.spmv(a.rowptr, a.col, a.val.astype(np.float32).astype(np.float64),
                              x_np)[E.stored_rows]
            else:
                full = L.spmv(a.rowptr, a.col, a.val.astype(np.float32).astype(np.float64), x_np)
            den = L.inf_norm(a.rowptr, q) * np.abs(x_np).max()
            den_a = L.inf_norm(a.rowptr, a.val) * np.abs(x_np).max()
            errors[name] = {"vs_oracle_same_q": float(np.abs(y - ref).max() / den),
                            "backward_error_eq5": float(np.abs(y - full).max() / den_a)}
        elif name.startswith("packed_csr"):  # rows in their own order
            A = r["A"]
            fmt = F.FMT_FP16 if A.fmt == 0 else F.FMT_E8MY
            q = P.quantized_values(a.rowptr, a.col, a.val, a.n, fmt, A.D)
            ref = L.spmv(a.rowptr, a.col, q, x_np)
            full = L.spmv(a.rowptr, a.col, a.val.astype(np.float32).astype(np.float64), x_np)
            den = L.inf_norm(a.rowptr, q) * np.abs(x_np).max()
            den_a = L.inf_norm(a.rowptr, a.val) * np.abs(x_np).max()
            errors[name] = {"vs_oracle_same_q": float(np.abs(y - ref).max() / den),
                            "backward_error_eq5": float(np.abs(y - full).max() / den_a)}
        else:
            E = P.encode(a.rowptr, a.col, a.val, a.n, a.m, F.FMT_E8MY, 22, 64, 256, 0)
            vdt = r["S"].value_dtype
            v32 = a.val.astype(np.float32)
            vals = (a.val if vdt == torch.float64 else
                    (v32.astype(np.float16) if vdt == torch.float16 else v32).astype(np.float64))
            ref = L.spmv(a.rowptr, a.col, vals, x_np)[E.stored_rows]
            full = L.spmv(a.rowptr, a.col, a.val, x_np)[E.stored_rows]
            den = L.inf_norm(a.rowptr, vals) * np.abs(x_np).max()
            errors[name] = {"vs_oracle_same_values": float(np.abs(y - ref).max() / den),
                            "backward_error_eq5": float(np.abs(y - full).max() / den)}
    for name, (m, xx, ys) in EXTRA_CHECKS.items():
        xd = xx.astype(np.float64)
        full = L.spmv(m.rowptr, m.col, m.val, xd)
        den = L.inf_norm(m.rowptr, m.val) * np.abs(xd).max()
        for var, (y, fmt, D) in ys.items():
            y = y.astype(np.float64)
            e = {"backward_error_eq5": float(np.abs(y - full).max() / den)}
            q = quantised(m, fmt, D)
            if q is not None:
                ref = L.spmv(m.rowptr, m.col, q, xd)
                e["vs_oracle_same_q"] = float(np.abs(y - ref).max() /
                                              (L.inf_norm(m.rowptr, q) * np.abs(xd).max()))
            errors[f"{name}.{var}"] = e
    return {"value": round(csr_bytes / dt / 1e9, 2), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{reps} float64 CSR SpMVs of the 7-point {round(a.n ** (1 / 3))}^3 "
                      f"Laplacian (FP16-quantised values) on {cores} host threads, "
                      f"{dt * 1e3:.1f} ms each, and {reps1} on one thread, {dt1 * 1e3:.1f} ms "
                      f"each; rate = the oracle's own CSR bytes ({csr_bytes} per product) "
                      f"per product time",
            "ms_per_spmv": round(dt * 1e3, 3),
            "single_thread": {"value": round(csr_bytes / dt1 / 1e9, 3), "unit": "GB/s",
                              "ms_per_spmv": round(dt1 * 1e3, 3), "cores": 1},
            "oracle_ms_over_gpu_ms": round(dt * 1e3 / H["ms"], 1),
            "errors": errors}


if __name__ == "__main__":
    main()
