"""Counter-based fault sampling.

Shot ``b`` of a run with key ``key`` is a pure function of (key, b): fault j
occurs iff word (j mod 4) of Philox4x32-10(key, ctr = (floor(j/4), b_lo, b_hi,
0)) is below floor(p_j * 2^32).  Philox4x32-10 is the counter-based generator
of Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11): ten rounds of two 32x32->64 multiplies with the multipliers
0xD2511F53 and 0xCD9E8D57, the key bumped by the Weyl constants 0x9E3779B9 and
0xBB67AE85 between rounds.  This implementation (vectorised numpy) is used only
to draw inputs; the decoder's own memory-strength generator is implemented
separately on each side.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: 4 uint32 arrays (broadcastable), key: 2 uint32 scalars/arrays.

    Returns a tuple of 4 uint32 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint32) for c in ctr)
    k0 = np.asarray(key[0], dtype=np.uint32)
    k1 = np.asarray(key[1], dtype=np.uint32)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = (k0 + _W0).astype(np.uint32)
                k1 = (k1 + _W1).astype(np.uint32)
            p0 = c0.astype(np.uint64) * _M0
            p1 = c2.astype(np.uint64) * _M1
            hi0 = (p0 >> _S32).astype(np.uint32)
            lo0 = (p0 & _MASK).astype(np.uint32)
            hi1 = (p1 >> _S32).astype(np.uint32)
            lo1 = (p1 & _MASK).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def split_key(key: int):
    key = int(key) & 0xFFFFFFFFFFFFFFFF
    return np.uint32(key & 0xFFFFFFFF), np.uint32(key >> 32)


def prior_thresholds(prior) -> np.ndarray:
    """floor(p * 2^32) per column, saturated to 2^32 - 1."""
    t = np.floor(np.asarray(prior, dtype=np.float64) * 4294967296.0)
    return np.minimum(t, 4294967295.0).astype(np.uint64)


def sample_faults(prior, key: int, shot0: int, count: int) -> np.ndarray:
    """uint8 [count, N] fault bits for shots shot0 .. shot0+count-1."""
    prior = np.asarray(prior, dtype=np.float64)
    n = prior.size
    nq = (n + 3) // 4
    shots = np.arange(shot0, shot0 + count, dtype=np.uint64)
    s_lo = (shots & _MASK).astype(np.uint32)[:, None]
    s_hi = (shots >> _S32).astype(np.uint32)[:, None]
    q = np.arange(nq, dtype=np.uint32)[None, :]
    zero = np.zeros((1, 1), dtype=np.uint32)
    words = philox4x32_10((q, s_lo, s_hi, zero), split_key(key))
    x = np.stack(words, axis=-1).reshape(count, nq * 4)[:, :n]
    return (x.astype(np.uint64) < prior_thresholds(prior)[None, :]).astype(np.uint8)


def syndromes(rows, cols, m: int, faults: np.ndarray) -> np.ndarray:
    """sigma = H F over GF(2) for a batch of fault vectors (uint8 [B, M])."""
    faults = np.asarray(faults, dtype=np.uint8)
    b = faults.shape[0]
    out = np.zeros((b, m), dtype=np.uint8)
    contrib = faults[:, cols]  # [B, nnz]
    for r in np.unique(rows):
        sel = rows == r
        out[:, r] = np.bitwise_xor.reduce(contrib[:, sel], axis=1)
    return out


def sample_batch(problem, key: int, shot0: int, count: int, chunk: int = 65536):
    """(faults, syndromes) for a contiguous range of shots, chunked."""
    fs, ss = [], []
    for s in range(shot0, shot0 + count, chunk):
        c = min(chunk, shot0 + count - s)
        f = sample_faults(problem.prior, key, s, c)
        fs.append(f)
        ss.append(syndromes(problem.rows, problem.cols, problem.m, f))
    if not fs:
        return (np.zeros((0, problem.n), np.uint8), np.zeros((0, problem.m), np.uint8))
    return np.concatenate(fs), np.concatenate(ss)


def sample_syndromes_sparse(problem, seed: int, count: int, chunk: int = 20000):
    """Fast sampler for large shot counts (input generation only).

    Per column j the number of shots containing fault j is Binomial(count, p_j)
    and those shots are a uniform subset; this yields the same distribution as
    independent Bernoulli(p_j) draws per (shot, column).  Returns
    (syndromes uint8 [count, M], fault shot/column lists).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    prior = problem.prior
    csr_ptr, csr_col = None, None
    # column -> rows
    order = np.argsort(problem.cols, kind="stable")
    ccols = problem.cols[order]
    crows = problem.rows[order]
    colptr = np.searchsorted(ccols, np.arange(problem.n + 1))
    k = rng.binomial(count, prior)
    shot_list, col_list = [], []
    for j in np.nonzero(k)[0]:
        s = rng.choice(count, size=int(k[j]), replace=False)
        shot_list.append(s)
        col_list.append(np.full(s.size, j, dtype=np.int64))
    shots = np.concatenate(shot_list) if shot_list else np.zeros(0, np.int64)
    fcols = np.concatenate(col_list) if col_list else np.zeros(0, np.int64)
    syn = np.zeros((count, problem.m), dtype=np.uint8)
    for s0 in range(0, count, chunk):
        s1 = min(count, s0 + chunk)
        sel = (shots >= s0) & (shots < s1)
        ss, cc = shots[sel] - s0, fcols[sel]
        deg = colptr[cc + 1] - colptr[cc]
        rep_s = np.repeat(ss, deg)
        starts = np.repeat(colptr[cc], deg)
        offs = np.arange(rep_s.size) - np.repeat(np.cumsum(deg) - deg, deg)
        rr = crows[starts + offs]
        cnt = np.bincount(rep_s * problem.m + rr, minlength=(s1 - s0) * problem.m)
        syn[s0:s1] = (cnt & 1).reshape(s1 - s0, problem.m).astype(np.uint8)
    del csr_ptr, csr_col
    return syn, (shots, fcols)
