"""Validity of bit-packed corrections, checked on the CPU.

A correction e of shot b is valid when H e = s_b over GF(2), the decoding
problem's constraint (paper Sec. 2.1).  The check here uses only the sparse
H (rows, cols), scipy's sparse product and numpy, so it shares nothing with
the HIP path and holds at any batch size.
"""
import numpy as np
import scipy.sparse as sp


def packed_positions(words, n):
    """(shot, column) of every set bit of packed words [B, ceil(n/32)] (entry k
    in bit k % 32 of word k // 32); asserts no bit past column n - 1 is set."""
    w = np.ascontiguousarray(words).view(np.uint32)
    r, q = np.nonzero(w)
    vals = w[r, q]
    rows, cols = [], []
    for bit in range(32):
        hit = ((vals >> np.uint32(bit)) & np.uint32(1)).astype(bool)
        rows.append(r[hit])
        cols.append(q[hit].astype(np.int64) * 32 + bit)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    assert (cols < n).all(), "bits past the last column are set"
    return rows, cols


def valid_shots(prob, corr_words, syn, chunk=200000):
    """bool [B]: H e_b = s_b (mod 2) for the packed corrections corr_words
    [B, ceil(N/32)] against the syndromes syn uint8 [B, M]."""
    b = corr_words.shape[0]
    h_t = sp.csr_matrix((np.ones(prob.nnz, np.int32), (prob.cols, prob.rows)), shape=(prob.n, prob.m))
    ok = np.empty(b, dtype=bool)
    for s0 in range(0, b, chunk):
        s1 = min(b, s0 + chunk)
        rows, cols = packed_positions(corr_words[s0:s1], prob.n)
        e = sp.csr_matrix((np.ones(rows.size, np.int32), (rows, cols)), shape=(s1 - s0, prob.n))
        he = (e @ h_t).toarray() & 1
        ok[s0:s1] = (he == (syn[s0:s1] != 0)).all(1)
    return ok
