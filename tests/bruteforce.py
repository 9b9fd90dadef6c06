"""Brute-force references for tiny decoding problems (tests only).

Exhaustive enumeration over all 2^N fault sets of the decoding problem of the
paper's Sec. 2.1: cost of F is sum_j w_j F_j (= -log Pr(F) up to a constant,
with w_j = log((1-p_j)/p_j)), validity is H F = sigma over GF(2).
"""
from __future__ import annotations

import numpy as np


def all_fault_sets(n: int) -> np.ndarray:
    idx = np.arange(1 << n, dtype=np.int64)
    return ((idx[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)


def valid_sets(h: np.ndarray, sigma: np.ndarray):
    fs = all_fault_sets(h.shape[1])
    syn = (fs.astype(np.int64) @ h.T.astype(np.int64)) % 2
    ok = (syn == np.asarray(sigma)[None, :]).all(axis=1)
    return fs[ok]


def min_marginals(h, sigma, w):
    """C_j(1) - C_j(0), with C_j(b) = min cost over valid F with F_j = b."""
    fs = valid_sets(h, sigma)
    cost = fs.astype(np.float64) @ np.asarray(w, dtype=np.float64)
    n = h.shape[1]
    out = np.zeros(n)
    for j in range(n):
        c1 = cost[fs[:, j] == 1]
        c0 = cost[fs[:, j] == 0]
        out[j] = (c1.min() if c1.size else np.inf) - (c0.min() if c0.size else np.inf)
    return out


def min_weight_solutions(h, sigma, w):
    fs = valid_sets(h, sigma)
    cost = fs.astype(np.float64) @ np.asarray(w, dtype=np.float64)
    best = cost.min()
    return fs[cost == best], best


def exact_marginal_llr(h, sigma, w):
    """log P(F_j = 0 | sigma) - log P(F_j = 1 | sigma) under Pr(F) ~ exp(-sum w F)."""
    fs = valid_sets(h, sigma)
    logp = -(fs.astype(np.float64) @ np.asarray(w, dtype=np.float64))
    mx = logp.max()
    pw = np.exp(logp - mx)
    out = np.zeros(h.shape[1])
    for j in range(h.shape[1]):
        out[j] = np.log(pw[fs[:, j] == 0].sum()) - np.log(pw[fs[:, j] == 1].sum())
    return out


def random_tree(rng, n_checks: int, min_check_degree: int = 2):
    """Random bipartite tree Tanner graph; every check has degree >= min_check_degree.

    Grown node by node: a new check hangs off an existing fault, a new fault
    off an existing check; checks left with too few faults get new leaf faults.
    Returns a dense H (M x N).
    """
    edges = []
    n_faults = 1
    checks = 0
    while checks < n_checks:
        if rng.random() < 0.5 or checks == 0:
            edges.append((checks, int(rng.integers(0, n_faults))))
            checks += 1
        else:
            edges.append((int(rng.integers(0, checks)), n_faults))
            n_faults += 1
    deg = np.zeros(checks, int)
    for i, _ in edges:
        deg[i] += 1
    for i in range(checks):
        while deg[i] < min_check_degree:
            edges.append((i, n_faults))
            n_faults += 1
            deg[i] += 1
    h = np.zeros((checks, n_faults), dtype=np.uint8)
    for i, j in edges:
        h[i, j] = 1
    # random relabelling of faults and checks keeps the CSR order non-trivial
    h = h[rng.permutation(checks)][:, rng.permutation(n_faults)]
    return h


def tree_diameter(h) -> int:
    m, n = h.shape
    adj = [[] for _ in range(m + n)]
    for i, j in zip(*np.nonzero(h)):
        adj[i].append(m + j)
        adj[m + j].append(i)

    def far(src):
        dist = {src: 0}
        stack = [src]
        while stack:
            u = stack.pop()
            for v in adj[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    stack.append(v)
        node = max(dist, key=dist.get)
        return node, dist[node]

    a, _ = far(m)
    _, d = far(a)
    return d
