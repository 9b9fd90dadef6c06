"""Pins of the oracle's binary16 mode (reduced-precision messages).

The mode runs Relay with every per-shot quantity held in IEEE binary16 and
every arithmetic result rounded to binary16, nearest-even; see the mode's
header in oracle/relay_oracle.c.  What fixes it here: the rounding function
against a second implementation (numpy's double -> float16 conversion) and
hand-picked values of the format; exact tree min-marginals with small
integer LLRs (no rounding can occur); equality with the FP32 decoder where
all arithmetic is exact in both; and one iteration on a path graph whose
values do round, recomputed step by step with numpy float16 arithmetic."""
import numpy as np
import pytest

import oracle
from tests import bruteforce as bf
from tests.conftest import RELAY_DEFAULT
from tests.test_oracle_pins import _coo, _prior_from_llr, _tree_case
from workloads import codes, sampling


def test_round_h16_matches_numpy_float16():
    rng = np.random.default_rng(0)
    xs = rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 5.5, 20000)
    for x in xs:
        with np.errstate(over="ignore"):
            ref = float(np.float16(x))
        got = oracle.round_h16(x)
        assert got == ref and np.signbit(got) == np.signbit(ref), x


@pytest.mark.parametrize("x,expect", [
    (1.0 / 3.0, 0.333251953125),          # 0x3555
    (65504.0, 65504.0), (65519.99, 65504.0), (65520.0, np.inf), (-1e9, -np.inf),
    (2049.0, 2048.0), (2051.0, 2052.0),   # ties to even at spacing 2
    (2.0 ** -24, 2.0 ** -24), (2.0 ** -25, 0.0), (3 * 2.0 ** -26, 2.0 ** -24),
    (0.1, 0.0999755859375), (-0.0, -0.0),
])
def test_round_h16_known_values(x, expect):
    got = oracle.round_h16(x)
    assert got == expect and np.signbit(got) == np.signbit(expect)


@pytest.mark.parametrize("seed", range(8))
def test_h16_tree_min_marginals_exact(seed):
    """Min-sum with gamma = 0 on a tree, T >= diameter: the marginals are the
    exact min-marginals C_j(1) - C_j(0) (small integers, exact in binary16)."""
    h, w, sigma = _tree_case(seed, 6)
    r, c = _coo(h)
    T = 2 * h.shape[1]
    tr = oracle.trace(h.shape[0], h.shape[1], r, c, _prior_from_llr(w), np.zeros(h.shape[1], np.float32), T,
                      sigma[None].astype(np.uint8), precision="h16")[0]
    expect = bf.min_marginals(h, sigma, w)
    np.testing.assert_array_equal(tr[T], expect.astype(np.float32))


@pytest.mark.parametrize("name", ["bb72", "bb144"])
def test_h16_equals_f32_where_arithmetic_is_exact(name):
    """Integer LLRs (w = 3), gamma = 0 in every leg and L = 512: every value
    is an integer of magnitude <= 2560, and those above 2048 are clipped to
    512 whether rounded or not, so both modes compute the same numbers."""
    code = codes.bb_code(name)
    p = codes.problem_from_dense(name, code.hx, 1.0 / (1.0 + np.exp(3.0)), code.logical)
    _, syn = sampling.sample_batch(codes.bb_problem(name, 0.08), 93, 0, 200)
    prm = dict(RELAY_DEFAULT, num_legs=6, num_solutions=2, gamma_first=0.0, gamma_lo=0.0, gamma_hi=0.0,
               llr_clip=512.0)
    a = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True)
    b = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True, precision="h16")
    assert np.abs(a["llr"]).max() > 64
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def _h16_reference(h, w, g, sigma, T, L=4096.0):
    """The binary16 mode's leg written out with numpy's float16 conversion as
    the rounding (each sum, difference or product formed in float64, exact for
    two binary16 operands, then converted once): Lambda(t) for t = 1..T."""
    f16 = np.float16

    def rnd(x):
        return f16(np.float64(x))

    def clip(x):
        return f16(min(max(float(x), -L), L))

    m, n = h.shape
    rows = [list(np.nonzero(h[i])[0]) for i in range(m)]
    Lam = [f16(x) for x in w]
    mu = {(i, j): f16(0) for i in range(m) for j in rows[i]}
    out = []
    for _ in range(T):
        nu = {(i, j): clip(rnd(np.float64(Lam[j]) - np.float64(mu[(i, j)]))) for i in range(m) for j in rows[i]}
        new = {}
        for i in range(m):
            for j in rows[i]:
                others = [k for k in rows[i] if k != j]
                neg = int(sigma[i]) ^ (sum(int(nu[(i, k)] < 0) for k in others) & 1)
                mag = min([abs(float(nu[(i, k)])) for k in others], default=np.inf)
                new[(i, j)] = clip(-mag if neg else mag)
        mu = new
        cur = []
        for j in range(n):
            a = rnd(np.float64(rnd(1.0 - np.float64(g[j]))) * np.float64(w[j]))
            b = rnd(np.float64(g[j]) * np.float64(clip(Lam[j])))
            acc = clip(rnd(np.float64(a) + np.float64(b)))
            for i in range(m):
                if (i, j) in mu:
                    acc = rnd(np.float64(acc) + np.float64(mu[(i, j)]))
            cur.append(acc)
        Lam = cur
        out.append(np.array(Lam, np.float32))
    return np.array(out)


@pytest.mark.parametrize("case", ["path", "cycle", "loopy"])
def test_h16_iterations_with_rounding_against_numpy_float16(case):
    """Twelve iterations of one leg on small graphs whose values round at
    every step (LLRs with many significant bits, memory strengths whose
    binary16 values make 1 - gamma round), against the leg written out with
    numpy float16 conversions."""
    rng = np.random.default_rng({"path": 1, "cycle": 2, "loopy": 3}[case])
    if case == "path":
        h = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    elif case == "cycle":
        h = np.array([[1, 1, 0, 0, 0], [0, 1, 1, 0, 0], [0, 0, 1, 1, 0], [0, 0, 0, 1, 1], [1, 0, 0, 0, 1]],
                     np.uint8)
    else:
        h = (rng.random((6, 10)) < 0.4).astype(np.uint8)
        h[0, :] = 1
    m, n = h.shape
    r, c = _coo(h)
    wd = rng.uniform(0.7, 9.3, n)
    prior = _prior_from_llr(wd)
    g32 = rng.uniform(0.05, 0.95, n).astype(np.float32)
    sigma = (rng.random(m) < 0.5).astype(np.uint8)
    T = 12
    tr = oracle.trace(m, n, r, c, prior, g32, T, sigma[None], precision="h16")[0]
    w16 = np.array([np.float16(np.log((1 - q) / q)) for q in prior])
    g16 = np.array([np.float16(x) for x in g32])
    ref = _h16_reference(h, w16, g16, sigma, T)
    np.testing.assert_array_equal(tr[1:], ref)
    exact = np.array([(1.0 - float(x)) for x in g16])
    assert (exact != np.array([float(np.float16(x)) for x in exact])).any()   # 1 - gamma rounds
