"""Decoding problems: bivariate-bicycle codes and a DEM-shaped synthetic matrix.

Everything here is input construction.  The decoding problem is the triple
(H, A, p) of paper Sec. 2.1 (the circuit-decoding-problem paragraph): H is the
M x N detector/check matrix, A the K x N logical action matrix, p the vector of
independent fault probabilities.

* Bivariate-bicycle (BB) codes, code-capacity noise: H is the X-check matrix
  HX = [A_poly | B_poly] of a BB code (the gross code family the paper
  benchmarks in Sec. 2.1, decoding-examples paragraph), faults are Z errors on
  the n data qubits with a uniform probability p, and the logical matrix is a
  basis of ker(HZ) modulo rowspace(HX) (X-type logical representatives, which
  detect every nontrivial Z-type logical).
* A DEM-shaped synthetic matrix standing in for the paper's 936 x 8784 gross
  circuit-level Z decoding matrix (Sec. 2.1, decoding-examples paragraph):
  13 rounds of 72 detectors, each fault touching 2-6 detectors inside a band of
  72 rows around its round.  The real DEM needs circuits and a DEM generator
  that are not available, so this synthetic matrix with the same shape, row
  count and sparsity structure stands in for it; its logical matrix is a dense
  random 12-row matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# GF(2) linear algebra (plain elimination on uint8 arrays)
# --------------------------------------------------------------------------


def gf2_rref(mat: np.ndarray):
    """Row-reduce a binary matrix over GF(2).

    Returns (R, pivots): R is the reduced row-echelon form (same shape, uint8)
    and pivots the list of pivot columns, one per nonzero row of R.
    """
    a = (np.asarray(mat, dtype=np.uint8) & 1).copy()
    rows, cols = a.shape
    pivots = []
    r = 0
    for c in range(cols):
        if r >= rows:
            break
        nz = np.nonzero(a[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + nz[0]
        if p != r:
            a[[r, p]] = a[[p, r]]
        others = np.nonzero(a[:, c])[0]
        others = others[others != r]
        if others.size:
            a[others] ^= a[r]
        pivots.append(c)
        r += 1
    return a, pivots


def gf2_rank(mat: np.ndarray) -> int:
    return len(gf2_rref(mat)[1])


def gf2_nullspace(mat: np.ndarray) -> np.ndarray:
    """Basis (rows) of {x : mat x = 0} over GF(2)."""
    a = np.asarray(mat, dtype=np.uint8) & 1
    n = a.shape[1]
    r, pivots = gf2_rref(a)
    free = [c for c in range(n) if c not in set(pivots)]
    basis = np.zeros((len(free), n), dtype=np.uint8)
    for k, f in enumerate(free):
        basis[k, f] = 1
        for row, pc in enumerate(pivots):
            if r[row, f]:
                basis[k, pc] = 1
    return basis


# --------------------------------------------------------------------------
# Bivariate-bicycle codes
# --------------------------------------------------------------------------


def _shift(n: int) -> np.ndarray:
    s = np.zeros((n, n), dtype=np.uint8)
    s[np.arange(n), (np.arange(n) + 1) % n] = 1
    return s


def _mat_pow(m: np.ndarray, e: int) -> np.ndarray:
    out = np.eye(m.shape[0], dtype=np.uint8)
    for _ in range(e):
        out = (out.astype(np.int64) @ m) % 2
    return out.astype(np.uint8)


def bb_polynomial(l: int, m: int, terms) -> np.ndarray:
    """Sum over GF(2) of monomials x^a y^b with x = S_l (x) I_m, y = I_l (x) S_m.

    ``terms`` is a list of ('x', a) / ('y', b) / ('1', 0) monomials.
    """
    x = np.kron(_shift(l), np.eye(m, dtype=np.uint8)).astype(np.uint8)
    y = np.kron(np.eye(l, dtype=np.uint8), _shift(m)).astype(np.uint8)
    acc = np.zeros((l * m, l * m), dtype=np.uint8)
    for var, e in terms:
        if var == "x":
            acc ^= _mat_pow(x, e)
        elif var == "y":
            acc ^= _mat_pow(y, e)
        elif var == "1":
            acc ^= np.eye(l * m, dtype=np.uint8)
        else:
            raise ValueError(var)
    return acc


@dataclass
class BBCode:
    name: str
    l: int
    m: int
    a_terms: list
    b_terms: list
    hx: np.ndarray = field(repr=False, default=None)
    hz: np.ndarray = field(repr=False, default=None)
    logical: np.ndarray = field(repr=False, default=None)  # rows: X-type logicals

    @property
    def n(self) -> int:
        return 2 * self.l * self.m

    @property
    def k(self) -> int:
        return self.n - gf2_rank(self.hx) - gf2_rank(self.hz)


# (l, m, A, B) of the four bivariate-bicycle codes used by the workloads.
BB_SPECS = {
    "bb72": (6, 6, [("x", 3), ("y", 1), ("y", 2)], [("y", 3), ("x", 1), ("x", 2)]),
    "bb90": (15, 3, [("x", 9), ("y", 1), ("y", 2)], [("1", 0), ("x", 2), ("x", 7)]),
    "bb144": (12, 6, [("x", 3), ("y", 1), ("y", 2)], [("y", 3), ("x", 1), ("x", 2)]),
    "bb288": (12, 12, [("x", 3), ("y", 2), ("y", 7)], [("y", 3), ("x", 1), ("x", 2)]),
}


def logical_basis(hx: np.ndarray, hz: np.ndarray) -> np.ndarray:
    """Rows spanning ker(hz) modulo rowspace(hx) (one row per logical qubit)."""
    ker = gf2_nullspace(hz)
    basis = [row for row in np.asarray(hx, dtype=np.uint8)]
    rank = gf2_rank(np.array(basis))
    chosen = []
    for v in ker:
        trial = np.array(basis + [v])
        r2 = gf2_rank(trial)
        if r2 > rank:
            basis.append(v)
            chosen.append(v)
            rank = r2
    return np.array(chosen, dtype=np.uint8).reshape(len(chosen), hx.shape[1])


def bb_code(name: str) -> BBCode:
    l, m, at, bt = BB_SPECS[name]
    a = bb_polynomial(l, m, at)
    b = bb_polynomial(l, m, bt)
    hx = np.concatenate([a, b], axis=1).astype(np.uint8)
    hz = np.concatenate([b.T, a.T], axis=1).astype(np.uint8)
    code = BBCode(name, l, m, at, bt, hx=hx, hz=hz)
    code.logical = logical_basis(hx, hz)
    return code


# --------------------------------------------------------------------------
# Problem container
# --------------------------------------------------------------------------


@dataclass
class Problem:
    """A decoding problem (H, A, p) with H stored as COO (row-major sorted)."""

    name: str
    m: int
    n: int
    rows: np.ndarray  # int32 [nnz]
    cols: np.ndarray  # int32 [nnz]
    prior: np.ndarray  # float64 [n]
    logical: np.ndarray  # uint8 [K, n]

    @property
    def nnz(self) -> int:
        return int(self.rows.size)

    def dense(self) -> np.ndarray:
        h = np.zeros((self.m, self.n), dtype=np.uint8)
        h[self.rows, self.cols] = 1
        return h

    def csr(self):
        """(rowptr, colidx) with columns ascending inside each row."""
        order = np.lexsort((self.cols, self.rows))
        r = self.rows[order]
        c = self.cols[order].astype(np.int32)
        rowptr = np.zeros(self.m + 1, dtype=np.int64)
        np.add.at(rowptr, r + 1, 1)
        return np.cumsum(rowptr), c


def problem_from_dense(name, h, prior, logical) -> Problem:
    h = np.asarray(h, dtype=np.uint8)
    r, c = np.nonzero(h)
    prior = np.broadcast_to(np.asarray(prior, dtype=np.float64), (h.shape[1],)).copy()
    return Problem(name, h.shape[0], h.shape[1], r.astype(np.int32), c.astype(np.int32),
                   prior, np.asarray(logical, dtype=np.uint8))


def bb_problem(name: str, p: float) -> Problem:
    """Code-capacity decoding problem on HX of a BB code with uniform prior p."""
    code = bb_code(name)
    return problem_from_dense(f"{name}_p{p}", code.hx, p, code.logical)


# --------------------------------------------------------------------------
# DEM-shaped synthetic matrix (936 detectors = 13 rounds x 72)
# --------------------------------------------------------------------------

DEM_WEIGHTS = np.array([2, 3, 4, 5, 6])
DEM_WEIGHT_P = np.array([0.35, 0.35, 0.15, 0.10, 0.05])


def dem_problem(m: int = 936, n: int = 8785, band: int = 72, seed: int = 9368785,
                logical_rows: int = 12, p_lo: float = 1e-4, p_hi: float = 1e-2) -> Problem:
    """Banded random matrix shaped like a circuit-level detector error model.

    Column j: weight w in {2..6} with probabilities (.35, .35, .15, .10, .05);
    round boundary rho uniform in {0..rounds} with rounds = m // band (a fault
    sits between detector rounds rho-1 and rho); rows drawn without
    replacement from the band [s, s + band) where
    s = clamp(band*rho - band/2, 0, m - band), so the bands cover every row;
    prior p_j = 10^U(log10 p_lo,
    log10 p_hi).  Every row is guaranteed nonempty (an empty row gets one
    extra entry from a random column of its band).  Logical matrix: dense
    Bernoulli(1/2) rows.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    rounds = m // band
    w = rng.choice(DEM_WEIGHTS, size=n, p=DEM_WEIGHT_P)
    rho = rng.integers(0, rounds + 1, size=n)
    start = np.clip(band * rho - band // 2, 0, m - band)
    rows, cols = [], []
    for j in range(n):
        rr = rng.choice(band, size=int(w[j]), replace=False) + start[j]
        rows.append(rr)
        cols.append(np.full(rr.size, j))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    present = np.zeros(m, dtype=bool)
    present[rows] = True
    extra_r, extra_c = [], []
    for i in np.nonzero(~present)[0]:
        cand = np.nonzero((start <= i) & (i < start + band))[0]
        extra_r.append(i)
        extra_c.append(int(rng.choice(cand)))
    if extra_r:
        rows = np.concatenate([rows, np.array(extra_r)])
        cols = np.concatenate([cols, np.array(extra_c)])
    order = np.lexsort((cols, rows))
    rows = rows[order].astype(np.int32)
    cols = cols[order].astype(np.int32)
    prior = 10.0 ** rng.uniform(np.log10(p_lo), np.log10(p_hi), size=n)
    logical = (rng.random((logical_rows, n)) < 0.5).astype(np.uint8)
    return Problem(f"dem{m}x{n}", m, n, rows, cols, prior, logical)


def dem_rounds_problem(m: int = 936, n: int = 8785, band: int = 72, seed: int = 9368785):
    """The DEM-shaped matrix of dem_problem with detector rounds made explicit
    for windowed decoding: rows of round r are [r*band, (r+1)*band), and the
    columns are reordered (stably) by the round of their first detector, so
    that the faults beginning in a range of rounds form a contiguous range of
    columns.  Returns (problem, first_round) with first_round[j] the round of
    column j's first detector (the number of rounds if the column is empty)."""
    p = dem_problem(m, n, band, seed)
    lo = np.full(n, m, dtype=np.int64)
    np.minimum.at(lo, p.cols, p.rows)
    first = lo // band
    order = np.argsort(first, kind="stable")
    new_of_old = np.empty(n, dtype=np.int64)
    new_of_old[order] = np.arange(n)
    cols = new_of_old[p.cols]
    srt = np.lexsort((cols, p.rows))
    prob = Problem(f"{p.name}_rounds", m, n, p.rows[srt].astype(np.int32), cols[srt].astype(np.int32),
                   p.prior[order], p.logical[:, order])
    return prob, first[order].astype(np.int32)
