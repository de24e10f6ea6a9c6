"""Shared test helpers: build both sides from the same seeded inputs."""
import numpy as np

from oracle import formats as F
from oracle import linalg as L
from oracle import packcsr as PC
from oracle import packsell as P
from paper_2604_13433_amd import workloads as W

# Parity bound for float32-accumulated products against the float64 oracle
# on the same quantised values, normalised by ||A_q||_inf ||x||_inf.
SPMV_TOL = 1e-6

FMTS = {"fp16": F.FMT_FP16, "e8my": F.FMT_E8MY, "fix": F.FMT_FIX}


def random_csr(seed, n, m, density=None, per_row=None, scale=1.0):
    """Random CSR with ~density*m (or ``per_row``) entries per row, a mix of
    near-diagonal and far columns so deltas of every size appear."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        k = per_row if per_row is not None else rng.binomial(m, density)
        k = min(k, m)
        if k == 0:
            continue
        ctr = (i * m) // max(n, 1)
        near = rng.integers(max(0, ctr - 40), min(m - 1, ctr + 40) + 1, size=k) if m else []
        far = rng.integers(0, m, size=k)
        pick = np.where(rng.random(k) < 0.7, near, far) if m else []
        c = np.unique(np.clip(pick, 0, m - 1))
        rows.append(np.full(c.size, i))
        cols.append(c)
    if rows:
        r = np.concatenate(rows)
        c = np.concatenate(cols)
    else:
        r = c = np.zeros(0, np.int64)
    v = rng.standard_normal(r.size) * scale
    return W.csr_from_triplets(n, m, r, c, v)


def oracle_product(a, fmt, D, x):
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, fmt, D)
    return L.spmv_multi(a.rowptr, a.col, q, x), q


def normalised_error(y, ref, a, q, x):
    den = L.inf_norm(a.rowptr, q) * float(np.max(np.abs(x))) if np.size(x) else 0.0
    err = float(np.max(np.abs(np.asarray(y, np.float64) - ref))) if np.size(y) else 0.0
    return err / den if den else err


def chunk_plan_from_words(E, T):
    """The expected plan of a product balanced over chunks of T words of a
    CSR-packed matrix E (the oracle's encoding), read off the word stream:
    lo[c] = the first row whose words start at or after word c*T
    (lo[n_chunks] = n), anchor[c] = the running column just before word c*T
    (the row's left offset when a row starts there)."""
    n_chunks = -(-E.n_words // T)
    starts = np.arange(n_chunks, dtype=np.int64) * T
    lo = np.empty(n_chunks + 1, dtype=np.int64)
    lo[:n_chunks] = np.searchsorted(E.wrowptr[:-1], starts, side="left")
    lo[n_chunks] = E.n
    anchor = np.zeros(n_chunks, dtype=np.int64)
    if n_chunks:
        after = PC.columns_after(E)
        r = PC.word_rows(E)[starts]
        head = E.wrowptr[r] == starts
        anchor[head] = PC.left_offset(r[head], E.k_left)
        anchor[~head] = after[starts[~head] - 1]
    return lo, anchor
