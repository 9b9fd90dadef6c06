"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test states what fixes it: a hand-worked example, a published
known-answer vector, a closed form, a textbook special case or brute force on
tiny inputs.  Together they are chosen so that a plausible slip in the oracle
(a dropped term, a wrong sign or index, a swapped gamma / 1-gamma, the wrong
iteration in the memory term, a wrong leg count) fails at least one of them.
"""
import os

import numpy as np
import pytest

import oracle
from tests import bruteforce as bf
from tests.conftest import RELAY_DEFAULT
from workloads import codes, sampling

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _coo(h):
    r, c = np.nonzero(h)
    return r.astype(np.int32), c.astype(np.int32)


def _prior_from_llr(w):
    """p with log((1-p)/p) = w (the oracle takes priors)."""
    return 1.0 / (1.0 + np.exp(np.asarray(w, dtype=np.float64)))


# ---------------------------------------------------------------- RNG -----


def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Salmon et al., SC'11)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr, key, exp = v[0:4], v[4:6], v[6:10]
        assert list(oracle.philox4x32_10(key, ctr)) == exp
        np_out = sampling.philox4x32_10([np.uint32(c) for c in ctr], key)
        assert [int(x) for x in np_out] == exp


def test_philox_two_implementations_agree():
    rng = np.random.default_rng(1)
    for _ in range(200):
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        a = oracle.philox4x32_10(key, ctr)
        b = sampling.philox4x32_10([np.uint32(c) for c in ctr], key)
        assert [int(x) for x in a] == [int(x) for x in b]


def test_gamma_distribution_and_formula():
    """gamma_{r,j} = lo + (hi-lo) * (x>>8) 2^-24 with x from Philox(seed; j/4, r)."""
    from scipy import stats

    seed, lo, hi = 0x52454C4159, -0.24, 0.66
    key = (seed & 0xFFFFFFFF, seed >> 32)
    vals = []
    for r in range(2, 12):
        for j in range(0, 400):
            g = oracle.gamma_f32(seed, r, j, lo, hi)
            x = int(sampling.philox4x32_10([np.uint32(j // 4), np.uint32(r), np.uint32(0),
                                            np.uint32(0)], key)[j % 4])
            u = np.float32(x >> 8) * np.float32(2.0 ** -24)
            expect = np.float32(lo) + (np.float32(hi) - np.float32(lo)) * u
            assert g == np.float32(expect)
            vals.append(float(g))
    vals = np.array(vals)
    assert vals.min() >= lo and vals.max() < hi
    assert stats.kstest((vals - lo) / (hi - lo), "uniform").pvalue > 1e-3


# ------------------------------------------------------- worked example ---


def _golden_path3():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "path3_worked_example.txt"))
            if l.strip() and not l.startswith("#")]
    return [(r[0], float(r[1]), int(r[2]), np.array([float(x) for x in r[3:]])) for r in rows]


def test_worked_example_path3():
    h = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    r, c = _coo(h)
    w = np.array([2.0, 3.0, 2.0])
    syn = np.array([[1, 1]], np.uint8)
    for name, gamma, t, expect in _golden_path3():
        if name == "minsum":
            tr = oracle.minsum_trace(2, 3, r, c, w, 3, syn)[0]
            tr2 = oracle.trace(2, 3, r, c, _prior_from_llr(w), 0.0, 3, syn, precision="f64")[0]
            np.testing.assert_allclose(tr2[t], expect, atol=1e-12)
        else:
            # priors whose FP32 LLRs are exactly w: compare in f64 with the
            # same exact w (prior -> LLR round trip is within 1e-15)
            tr = oracle.trace(2, 3, r, c, _prior_from_llr(w), gamma, 3, syn, precision="f64")[0]
            np.testing.assert_allclose(tr[t], expect, atol=1e-12)
            continue
        np.testing.assert_array_equal(tr[t], expect.astype(np.float32))


# ------------------------------------------------------------- trees ------


def _tree_case(seed, n_checks):
    rng = np.random.default_rng(seed)
    h = bf.random_tree(rng, n_checks)
    n = h.shape[1]
    w = rng.integers(1, 10, n).astype(np.float64)
    sigma = (rng.random(h.shape[0]) < 0.5).astype(np.uint8)
    return h, w, sigma


@pytest.mark.parametrize("seed", range(12))
def test_tree_min_marginals_exact(seed):
    """Min-sum is exact max-product on trees: Lambda_j = C_j(1) - C_j(0).

    Relay with gamma = 0 reduces to min-sum (Sec. 2.3: gamma_j = 0 recovers
    MinSum BP); with integer LLRs every FP32 operation is exact, so the
    agreement with brute force is bit-exact.
    """
    h, w, sigma = _tree_case(seed, n_checks=int(4 + seed % 5))
    n = h.shape[1]
    if n > 18:
        pytest.skip("tree too large for brute force")
    r, c = _coo(h)
    T = bf.tree_diameter(h) + 2
    mm = bf.min_marginals(h, sigma, w)
    assert np.isfinite(mm).all()
    # exact LLRs: pass w through the minsum trace (takes LLRs directly) and
    # through the Relay trace with gamma = 0 in f64 (priors round-trip to w)
    ms = oracle.minsum_trace(h.shape[0], n, r, c, w, T, sigma[None])[0, T]
    np.testing.assert_array_equal(ms, mm.astype(np.float32))
    rl = oracle.trace(h.shape[0], n, r, c, _prior_from_llr(w), 0.0, T, sigma[None],
                      precision="f64")[0, T]
    np.testing.assert_allclose(rl, mm, atol=1e-9)


@pytest.mark.parametrize("seed", range(12, 24))
def test_tree_hard_decision_is_min_weight(seed):
    """On trees with a unique minimum, the Relay decision is that minimum."""
    h, w, sigma = _tree_case(seed, n_checks=int(4 + seed % 5))
    n = h.shape[1]
    if n > 18:
        pytest.skip("tree too large for brute force")
    sols, best = bf.min_weight_solutions(h, sigma, w)
    if len(sols) != 1:
        pytest.skip("minimum not unique")
    r, c = _coo(h)
    prm = dict(RELAY_DEFAULT, num_legs=1, iters_first=bf.tree_diameter(h) + 2,
               gamma_first=0.0)
    out = oracle.decode(h.shape[0], n, r, c, _prior_from_llr(w), prm, sigma[None],
                        precision="f64")
    assert out["conv"][0] == 1
    np.testing.assert_array_equal(out["corr"][0], sols[0])
    assert out["weight"][0] == pytest.approx(best, abs=1e-9)


@pytest.mark.parametrize("seed", range(6))
def test_tree_sumproduct_marginals(seed):
    """Textbook: sum-product is exact on trees (FP64, 1e-10)."""
    rng = np.random.default_rng(100 + seed)
    h = bf.random_tree(rng, 5 + seed % 3)
    n = h.shape[1]
    if n > 16:
        pytest.skip("tree too large")
    w = rng.uniform(0.5, 4.0, n)
    sigma = (rng.random(h.shape[0]) < 0.5).astype(np.uint8)
    r, c = _coo(h)
    T = bf.tree_diameter(h) + 2
    sp = oracle.sumproduct_trace(h.shape[0], n, r, c, w, T, sigma[None])[0, T]
    np.testing.assert_allclose(sp, bf.exact_marginal_llr(h, sigma, w), atol=1e-10)


# ------------------------------------------------------ memory term -------


@pytest.mark.parametrize("gamma", [0.125, 0.3, -0.2])
@pytest.mark.parametrize("sigma", [0, 1])
def test_two_fault_memory_fixed_point(gamma, sigma):
    """One check of degree two: closed-form fixed point of the memory recurrence.

    With one check and faults a, b: mu_a(t) = s nu_b(t-1), nu_b = lambda_b
    (one neighbour), lambda(t) = (1-g) w + g Lambda(t-1), s = (-1)^sigma.  The
    fixed point solves (1-g) lambda_a = (1-g) w_a + g s lambda_b (and a<->b),
    Lambda_a = lambda_a + s lambda_b.  A swapped g / 1-g, a memory term using
    Lambda(t) or lambda(0) = Lambda, or a lost syndrome sign all move it.
    """
    h = np.array([[1, 1]], np.uint8)
    r, c = _coo(h)
    w = np.array([2.0, 3.5])
    s = -1.0 if sigma else 1.0
    a = np.array([[1 - gamma, -gamma * s], [-gamma * s, 1 - gamma]])
    lam = np.linalg.solve(a, (1 - gamma) * w)
    expect = np.array([lam[0] + s * lam[1], lam[1] + s * lam[0]])
    tr = oracle.trace(1, 2, r, c, _prior_from_llr(w), gamma, 400,
                      np.array([[sigma]], np.uint8), precision="f64")[0]
    np.testing.assert_allclose(tr[-1], expect, rtol=1e-9)


# --------------------------------------------------- gamma = 0 => BP ------


def test_gamma_zero_relay_equals_naive_minsum():
    """gamma = 0, one leg is min-sum BP (Sec. 2.3): the Relay iteration with
    nu = Lambda - mu and the separately written min-sum with explicit
    leave-one-out sums agree bit-exactly while every value is an integer
    below 2^24 (no rounding on either side)."""
    code = codes.bb_code("bb72")
    r, c = _coo(code.hx)
    rng = np.random.default_rng(5)
    w = np.full(72, 3.0)
    syn = (rng.random((8, 36)) < 0.3).astype(np.uint8)
    T = 7
    ms = oracle.minsum_trace(36, 72, r, c, w, T, syn)
    rl = oracle.trace(36, 72, r, c, _prior_from_llr(w), 0.0, T, syn, precision="f64")
    assert np.abs(ms).max() < 2 ** 24
    np.testing.assert_array_equal(rl.astype(np.float32), ms)


# ---------------------------------------------------- invariants ----------


def test_zero_syndrome_converges_at_first_iteration():
    p = codes.bb_problem("bb144", 0.04)
    syn = np.zeros((3, p.m), np.uint8)
    out = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, RELAY_DEFAULT, syn)
    assert (out["conv"] == 1).all() and (out["iters"] == 1).all() and (out["legs"] == 1).all()
    assert out["corr"].sum() == 0 and (out["weight"] == 0).all()


def test_leg_arithmetic_unsatisfiable_syndrome():
    """R counts every leg: 80 + 60 (R-1) iterations at most; for R = 301 that is
    18080 iterations = the paper's 36160-cycle maximum at 2 cycles/iteration
    (Sec. 7, real-time paragraph, and the appendix on Relay resources)."""
    code = codes.bb_code("bb72")
    h = np.vstack([code.hx, np.zeros((1, 72), np.uint8)])  # a row no fault touches
    r, c = _coo(h)
    syn = np.zeros((1, 37), np.uint8)
    syn[0, 36] = 1
    prm = dict(RELAY_DEFAULT, num_legs=301)
    out = oracle.decode(37, 72, r, c, np.full(72, 0.04), prm, syn)
    assert out["conv"][0] == 0
    assert out["iters"][0] == 18080 and 2 * out["iters"][0] == 36160
    assert out["legs"][0] == 301
    prm = dict(RELAY_DEFAULT, num_legs=301, max_total_iters=500)
    out = oracle.decode(37, 72, r, c, np.full(72, 0.04), prm, syn)
    assert out["iters"][0] == 500 and out["legs"][0] == 1 + (500 - 80 + 59) // 60


def test_degree_one_check_sends_clipped_message():
    """min over an empty set is +inf, saturated at L: a degree-1 check sends
    (-1)^sigma L, forcing its fault to sigma."""
    h = np.array([[1, 0], [1, 1]], np.uint8)
    r, c = _coo(h)
    w = np.array([2.0, 2.0])
    tr = oracle.trace(2, 2, r, c, _prior_from_llr(w), 0.0, 1, np.array([[1, 0]], np.uint8),
                      precision="f64")[0]
    # Lambda_0(1) = w0 + mu_{c0}(=-L) + mu_{c1}(= +nu_1 = 2)
    assert tr[1, 0] == pytest.approx(-(2.0 ** 64), rel=1e-12)


def test_validity_and_weight_on_small_loopy_graphs():
    rng = np.random.default_rng(7)
    for trial in range(30):
        m, n = 6, 12
        h = (rng.random((m, n)) < 0.3).astype(np.uint8)
        for j in range(n):
            if not h[:, j].any():
                h[rng.integers(0, m), j] = 1
        w = rng.integers(1, 6, n).astype(np.float64)
        f = (rng.random(n) < 0.2).astype(np.uint8)
        sigma = (h.astype(int) @ f) % 2
        r, c = _coo(h)
        out = oracle.decode(m, n, r, c, _prior_from_llr(w), RELAY_DEFAULT,
                            sigma[None].astype(np.uint8), precision="f64")
        if out["conv"][0]:
            assert ((h.astype(int) @ out["corr"][0]) % 2 == sigma).all()
            _, best = bf.min_weight_solutions(h, sigma, w)
            assert out["weight"][0] >= best - 1e-9


def test_single_faults_decode_on_bb_codes():
    for name in ("bb72", "bb144"):
        code = codes.bb_code(name)
        p = codes.bb_problem(name, 0.04)
        f = np.eye(p.n, dtype=np.uint8)
        syn = sampling.syndromes(p.rows, p.cols, p.m, f)
        out = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, RELAY_DEFAULT, syn)
        assert (out["conv"] == 1).all()
        resid = (f ^ out["corr"]).astype(int)
        assert not ((code.logical.astype(int) @ resid.T) % 2).any()


def test_batch_order_invariance_and_determinism():
    p = codes.bb_problem("bb72", 0.06)
    _, syn = sampling.sample_batch(p, 77, 0, 300)
    a = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, RELAY_DEFAULT, syn)
    perm = np.random.default_rng(0).permutation(300)
    b = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, RELAY_DEFAULT, syn[perm], threads=3)
    for k in a:
        np.testing.assert_array_equal(a[k][perm], b[k])


def test_bb_code_parameters():
    for name, k in (("bb72", 12), ("bb90", 8), ("bb144", 12), ("bb288", 12)):
        code = codes.bb_code(name)
        assert code.k == k
        assert not ((code.hx.astype(int) @ code.hz.T.astype(int)) % 2).any()
        assert (code.hx.sum(1) == 6).all() and (code.hx.sum(0) == 3).all()
        assert code.logical.shape == (k, code.n)
        assert not ((code.hz.astype(int) @ code.logical.T.astype(int)) % 2).any()
        stacked = np.vstack([code.hx, code.logical])
        assert codes.gf2_rank(stacked) == codes.gf2_rank(code.hx) + k


def test_dem_generator_statistics():
    p = codes.dem_problem()
    h = p.dense()
    assert (p.m, p.n) == (936, 8785)
    assert h.sum(1).min() >= 1
    cw = np.bincount(h.sum(0), minlength=7)[2:7] / p.n
    np.testing.assert_allclose(cw, [0.35, 0.35, 0.15, 0.10, 0.05], atol=0.02)
    assert 26500 < p.nnz < 28800
    assert 1e-4 <= p.prior.min() and p.prior.max() <= 1e-2


@pytest.mark.parametrize("anchor", [0, 1])
def test_leg_chaining_fixed_point(anchor):
    """Relay chaining (Sec. 2.3): leg r >= 2 starts from the previous leg's
    final marginals, lambda^{(r)}(0) = Lambda^{(r-1)}(T) (anchor 0), or keeps
    lambda(0) = w (anchor 1).  On one degree-2 check plus an unsatisfiable
    empty row (no leg ever converges), each long leg reaches the closed-form
    fixed point of the memory recurrence with its own gamma_{r,j} and its own
    anchor lambda(0): leg 1 from w, leg 2 from the leg-1 fixed point."""
    h = np.array([[1, 1], [0, 0]], np.uint8)
    r, c = _coo(h)
    w = np.array([2.0, 3.5])
    syn = np.array([[1, 1]], np.uint8)
    s = -1.0
    seed, lo, hi, g1 = 0xABCDEF, 0.05, 0.35, 0.125
    prm = dict(RELAY_DEFAULT, num_legs=2, iters_first=400, iters_leg=400, gamma_first=g1,
               gamma_lo=lo, gamma_hi=hi, seed=seed, anchor=anchor)
    out = oracle.decode(2, 2, r, c, _prior_from_llr(w), prm, syn, precision="f64",
                        want_llr=True)
    assert out["conv"][0] == 0 and out["iters"][0] == 800 and out["legs"][0] == 2

    def fixed_point(gam, lam0):
        a = np.array([[1 - gam[0], -gam[0] * s], [-gam[1] * s, 1 - gam[1]]])
        lam = np.linalg.solve(a, (1 - gam) * lam0)
        return np.array([lam[0] + s * lam[1], lam[1] + s * lam[0]])

    leg1 = fixed_point(np.array([g1, g1]), w)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    g2 = []
    for j in range(2):
        x = int(sampling.philox4x32_10([np.uint32(j // 4), np.uint32(2), np.uint32(0),
                                        np.uint32(0)], key)[j % 4])
        lo32, hi32 = float(np.float32(lo)), float(np.float32(hi))  # parameters are FP32
        g2.append(lo32 + (hi32 - lo32) * (x >> 8) * 2.0 ** -24)
    leg2 = fixed_point(np.array(g2), leg1 if anchor == 0 else w)
    np.testing.assert_allclose(out["llr"][0], leg2, rtol=1e-9)


# --------------------------------------------------------- learned first leg


def test_uniform_gamma1_equals_gamma_first():
    """A per-column leg-1 gamma vector filled with gamma_first is the paper's
    decoder exactly."""
    p = codes.bb_problem("bb72", 0.06)
    _, syn = sampling.sample_batch(p, 41, 0, 200)
    prm = dict(RELAY_DEFAULT, num_legs=8, num_solutions=2)
    a = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True)
    g1 = np.full(p.n, np.float32(prm["gamma_first"]), np.float32)
    b = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True, gamma1=g1)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("anchor", [0, 1])
def test_prior_scale_is_a_homogeneous_rescaling(anchor):
    """Min-sum with memory is positively homogeneous in the initial LLRs (min,
    signs, sums, products with gamma and the clip at 2^64 far away all commute
    with scaling), and scaling by a power of two is exact in floating point:
    with scale = 2 every decision, leg, iteration count and solution weight
    equals scale = 1, and the final marginals are exactly doubled.  A learned
    per-column gamma in leg 1 changes nothing in this."""
    p = codes.bb_problem("bb90", 0.06)
    _, syn = sampling.sample_batch(p, 43, 0, 200)
    prm = dict(RELAY_DEFAULT, num_legs=6, num_solutions=2, anchor=anchor)
    g1 = np.random.default_rng(4).uniform(-0.2, 0.6, p.n).astype(np.float32)
    a = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True, gamma1=g1)
    b = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True, gamma1=g1,
                      scale=2.0)
    for k in ("corr", "conv", "legs", "iters", "weight"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(b["llr"], np.float32(2.0) * a["llr"])


def test_learned_gamma1_changes_the_first_leg_only():
    """gamma1 enters leg 1 only: with one leg, the decode equals a leg-1 trace
    with per-column gamma (a different code path of the oracle) run to the
    first convergence."""
    p = codes.bb_problem("bb72", 0.05)
    _, syn = sampling.sample_batch(p, 47, 0, 60)
    g1 = np.random.default_rng(5).uniform(0.0, 0.5, p.n).astype(np.float32)
    T = 40
    prm = dict(RELAY_DEFAULT, num_legs=1, iters_first=T)
    out = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True, gamma1=g1,
                        scale=0.75)
    tr = oracle.trace(p.m, p.n, p.rows, p.cols, p.prior, g1, T, syn, scale=0.75)
    h = p.dense().astype(np.int64)
    for b in range(len(syn)):
        f = (tr[b, 1:] < 0).astype(np.int64)             # decisions after t = 1..T
        ok = np.nonzero(((f @ h.T) % 2 == (syn[b] != 0)).all(1))[0]
        t_stop = ok[0] + 1 if ok.size else T
        assert out["iters"][b] == t_stop
        assert out["conv"][b] == (1 if ok.size else 0)
        np.testing.assert_array_equal(out["llr"][b], tr[b, t_stop])
        np.testing.assert_array_equal(out["corr"][b], (tr[b, t_stop] < 0).astype(np.uint8))


# ------------------------------------------------ S > 1 solution selection


def _events_from_s_runs(h, w32, syn, prm, k_max, **kw):
    """Convergence events 1..k_max of every shot, read off decodes with
    S = 1..k_max.  The trajectory of a decode does not depend on S until it
    stops, so the run with S = k ends at the k-th convergence event, if there
    is one, and its final marginals give that event's decision
    F^(k) = [Lambda < 0].  Event k exists iff F^(k) satisfies the syndrome and
    the S = k run went past where the S = k-1 run stopped.  Returns, per
    shot, the list of (F^(k), W^(k)) with W^(k) = sum_j F^(k)_j w_j in FP64,
    and the outputs of every run."""
    outs = []
    for k in range(1, k_max + 1):
        outs.append(oracle.decode(h.shape[0], h.shape[1], *_coo(h), kw["prior"],
                                  dict(prm, num_solutions=k), syn, want_llr=True))
    hh = h.astype(np.int64)
    events = []
    for b in range(syn.shape[0]):
        ev = []
        for k in range(k_max):
            f = (outs[k]["llr"][b] < 0).astype(np.uint8)
            ok = ((hh @ f) % 2 == (syn[b] != 0)).all()
            past = k == 0 or outs[k]["iters"][b] > outs[k - 1]["iters"][b]
            if not (ok and past):
                break
            ev.append((f, float(np.sum(f.astype(np.float64) * w32.astype(np.float64)))))
        events.append(ev)
    return events, outs


def _check_selection(events, outs, k_max):
    """The S = k output is the earliest lowest-weight solution among events
    1..k (reading R7: lowest W, ties kept by the earliest), at that weight;
    the kept weight never increases with k.  Returns how many (shot, k) cases
    distinguish 'keep the lowest' from 'keep the last' and 'earliest on ties'
    from 'latest on ties'."""
    n_last, n_tie = 0, 0
    for b, ev in enumerate(events):
        prev_w = np.inf
        for k in range(1, k_max + 1):
            out = outs[k - 1]
            n_k = min(k, len(ev))
            assert out["conv"][b] == (1 if n_k else 0)
            if not n_k:
                continue
            ws = [e[1] for e in ev[:n_k]]
            best = int(np.argmin(ws))                 # first index of the minimum
            np.testing.assert_array_equal(out["corr"][b], ev[best][0])
            assert out["weight"][b] == ws[best]
            assert ws[best] <= prev_w
            prev_w = ws[best]
            if not np.array_equal(ev[best][0], ev[n_k - 1][0]):
                n_last += 1
            last_min = n_k - 1 - int(np.argmin(ws[::-1]))
            if last_min != best and not np.array_equal(ev[best][0], ev[last_min][0]):
                n_tie += 1
    return n_last, n_tie


def test_s_solutions_keep_the_earliest_lowest_weight_bb72():
    """Selection among S > 1 solutions on [[72,12,6]], R = 20.  Under the
    paper's chaining a leg that starts from the marginals of a converged leg
    converges again, to the same decision, at its first iteration, so the
    rule shows only where later legs find other solutions: with the prior
    anchor at p = 0.08 both rival rules (keep the last solution; keep the
    latest of equal weight) give a different output on some shot."""
    for p_, anchor, shots in ((0.06, 0, 200), (0.08, 1, 800)):
        p = codes.bb_problem("bb72", p_)
        _, syn = sampling.sample_batch(p, (1 << 32) | 6, 0, shots)
        w32 = np.full(p.n, np.float32(np.log((1 - p_) / p_)), np.float32)
        events, outs = _events_from_s_runs(p.dense(), w32, syn, dict(RELAY_DEFAULT, anchor=anchor), 5,
                                           prior=p.prior)
        n_last, n_tie = _check_selection(events, outs, 5)
        assert sum(len(e) == 5 for e in events) > shots // 2
        if anchor == 1:
            assert n_last > 0 and n_tie > 0


def test_s_solutions_on_small_loopy_graphs():
    """The same selection rule on random loopy graphs with unequal integer
    weights and the prior anchor, where later legs often find other
    solutions: both rival rules fail on some shot."""
    tot_last, tot_tie = 0, 0
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        m, n = 8, 16
        h = (rng.random((m, n)) < 0.3).astype(np.uint8)
        for j in range(n):
            if not h[:, j].any():
                h[rng.integers(0, m), j] = 1
        w = rng.integers(1, 5, n).astype(np.float64)
        f = (rng.random((200, n)) < 0.2).astype(np.uint8)
        syn = ((f.astype(np.int64) @ h.T) % 2).astype(np.uint8)
        prm = dict(RELAY_DEFAULT, num_legs=12, iters_first=20, iters_leg=15, anchor=1)
        events, outs = _events_from_s_runs(h, w.astype(np.float32), syn, prm, 4,
                                           prior=_prior_from_llr(w))
        n_last, n_tie = _check_selection(events, outs, 4)
        tot_last += n_last
        tot_tie += n_tie
    assert tot_last > 20 and tot_tie > 10


# ------------------------------------------------- weight <= 3 on [[72,12,6]]


def test_weight_at_least_min_weight_bb72():
    """Validity and weight against the exact minimum on [[72,12,6]]: for
    syndromes of random faults of weight <= 3, every fault set of weight <= 3
    is enumerated (1 + 72 + 2556 + 59640 sets), so the least weight among the
    enumerated solutions is the minimum weight of the syndrome.  A converged
    correction satisfies H F = sigma and weighs at least that much."""
    from itertools import combinations

    p = codes.bb_problem("bb72", 0.05)
    h = p.dense().astype(np.int64)
    colmask = (h * (1 << np.arange(p.m, dtype=np.int64))[:, None]).sum(0)   # syndrome bits per column
    best = {0: 0}
    for k in (1, 2, 3):
        for cset in combinations(range(p.n), k):
            s = 0
            for j in cset:
                s ^= int(colmask[j])
            best.setdefault(s, k)
    rng = np.random.default_rng(3)
    f = np.zeros((600, p.n), np.uint8)
    for b in range(600):
        f[b, rng.choice(p.n, rng.integers(1, 4), replace=False)] = 1
    syn = ((f.astype(np.int64) @ h.T) % 2).astype(np.uint8)
    out = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, dict(RELAY_DEFAULT, num_solutions=3), syn)
    assert out["conv"].mean() > 0.9
    for b in range(600):
        if not out["conv"][b]:
            continue
        assert ((h @ out["corr"][b]) % 2 == syn[b]).all()
        s = int((syn[b].astype(np.int64) << np.arange(p.m, dtype=np.int64)).sum())
        assert int(out["corr"][b].sum()) >= best[s]


# ------------------------------------------------ BB translation symmetry


@pytest.mark.parametrize("name", ["bb72", "bb90"])
def test_bb_translation_equivariance(name):
    """Translations (u, v) -> (u + a, v + b) of Z_l x Z_m commute with A and B
    (polynomials in the commuting shifts x, y), so they permute the checks and
    both halves of the faults of HX = [A | B] and leave H invariant.  With
    integer channel LLRs (w = 3), gamma = 0 in every leg and the clip at
    L = 2^20 (a marginal then stays below 4 L = 2^22 in magnitude) all
    arithmetic is exact, so decoding commutes with the permutation bit for bit: the
    decision, convergence, legs, iterations, weight and marginals of a
    translated syndrome are the translated ones."""
    code = codes.bb_code(name)
    l, m = code.l, code.m
    prior = 1.0 / (1.0 + np.exp(3.0))
    p = codes.problem_from_dense(name, code.hx, prior, code.logical)
    prm = dict(RELAY_DEFAULT, num_legs=6, num_solutions=2, gamma_first=0.0, gamma_lo=0.0, gamma_hi=0.0,
               llr_clip=2.0 ** 20)
    _, syn = sampling.sample_batch(codes.bb_problem(name, 0.08), 91, 0, 150)
    base = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn, want_llr=True)
    assert np.all(np.isin(base["llr"], np.round(base["llr"])))        # exact integer arithmetic
    for (a, b) in ((1, 0), (0, 1), (2, 1)):
        q = np.arange(l * m)
        t = ((q // m + a) % l) * m + (q % m + b) % m                   # check / half-column map
        tcol = np.concatenate([t, l * m + t])
        assert ((code.hx[np.ix_(t, tcol)] == code.hx)).all()
        syn_t = np.zeros_like(syn)
        syn_t[:, t] = syn
        out = oracle.decode(p.m, p.n, p.rows, p.cols, p.prior, prm, syn_t, want_llr=True)
        for key in ("conv", "legs", "iters", "weight"):
            np.testing.assert_array_equal(out[key], base[key])
        np.testing.assert_array_equal(out["corr"][:, tcol], base["corr"])
        np.testing.assert_array_equal(out["llr"][:, tcol], base["llr"])
