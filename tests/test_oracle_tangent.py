"""Pins of the oracle's tangent of one leg (forward-mode derivative of
Lambda(T) in the memory strengths gamma_j and the channel-LLR scale s, along
the FP32 trajectory; header of ro_tangent_f32 in oracle/relay_oracle.c).

What fixes it here, other than itself:
  * its FP32 values are the leg's own trace, bit for bit;
  * the scale direction: with no clip reached, every update of paper Sec. 2.3
    is positively homogeneous of degree one in (w', Lambda, mu), so Lambda(T)
    = A w' for the trajectory's fixed choices and dLambda(T)/ds = Lambda(T)/s
    (Euler's theorem) -- at the full training depth T = 60 too;
  * the gamma directions: central differences of the FP64 oracle (a separate
    code path, ro_trace_f64), on shots whose FP32 and FP64 trajectories agree
    and entries whose one-sided differences agree (no kink inside the
    stencil), with and without a clip that saturates.
Shots are selected by conditioning, not by result: a shot whose FP32 trace
departs from the FP64 trace by more than 1e-5 (relative, at any iteration)
follows different arithmetic and has no common derivative to compare."""
import numpy as np
import pytest

import oracle
from workloads import codes, sampling


def _case(b=64, seed=13, lo=0.05, hi=0.2):
    prob = codes.bb_problem("bb144", 0.04)
    _, syn = sampling.sample_batch(prob, (5 << 32) | seed, 0, b)
    gamma = np.random.default_rng(seed).uniform(lo, hi, prob.n).astype(np.float32)
    return prob, syn, gamma


def _well_conditioned(prob, syn, gamma, t_iters, scale=1.0, llr_clip=2.0 ** 64, tol=1e-5):
    t64 = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma.astype(np.float64),
                       t_iters, syn, scale=scale, precision="f64", llr_clip=llr_clip)
    t32 = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, t_iters, syn,
                       scale=scale, llr_clip=llr_clip).astype(np.float64)
    rel = (np.abs(t64 - t32) / np.maximum(np.abs(t64), 1.0)).reshape(len(syn), -1).max(axis=1)
    return rel < tol


@pytest.mark.parametrize("t_iters", [12, 60])
def test_tangent_values_are_the_trace(t_iters):
    prob, syn, gamma = _case(b=16)
    ref = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, t_iters, syn, scale=0.9)
    lam, _ = oracle.tangent(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, t_iters, syn,
                            np.zeros(prob.n), 1.0, scale=0.9)
    np.testing.assert_array_equal(lam, ref[:, t_iters])


@pytest.mark.parametrize("t_iters", [12, 60])
def test_scale_tangent_is_lambda_over_s(t_iters):
    """dLambda(T)/ds = Lambda(T)/s on shots that stay well-conditioned and
    below the clip (degree-one homogeneity of the min-sum leg)."""
    prob, syn, gamma = _case()
    s = 0.9
    lam, dl = oracle.tangent(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, t_iters, syn,
                             np.zeros(prob.n), 1.0, scale=s)
    tr = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, t_iters, syn, scale=s)
    below = np.abs(tr).reshape(len(syn), -1).max(axis=1) < 2.0 ** 60
    sel = below & _well_conditioned(prob, syn, gamma, t_iters, scale=s, tol=1e-4)
    assert sel.sum() >= 10, sel.sum()
    ref = lam[sel].astype(np.float64) / s
    err = np.abs(dl[sel] - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < 1e-4, err.max()
    # the gamma part of the direction contributes nothing at t = 1 (clip(Lambda(0)) = w')
    lam1, dl1 = oracle.tangent(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, 1, syn,
                               np.ones(prob.n), 0.0, scale=s)
    assert np.all(dl1 == 0.0)


@pytest.mark.parametrize("llr_clip", [2.0 ** 64, 20.0, 3.0])
def test_gamma_tangent_matches_fp64_central_differences(llr_clip):
    prob, syn, gamma = _case()
    t_iters, hh = 12, 1e-6
    g64 = gamma.astype(np.float64)
    agree = _well_conditioned(prob, syn, gamma, t_iters, llr_clip=llr_clip)
    assert agree.sum() >= 32, agree.sum()

    def lam64(g):
        return oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, g, t_iters, syn,
                            precision="f64", llr_clip=llr_clip)[:, t_iters]

    f0 = lam64(g64)
    checked = 0
    for j in range(0, prob.n, 7):
        d = np.zeros(prob.n)
        d[j] = 1.0
        _, dl = oracle.tangent(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, t_iters, syn, d,
                               0.0, llr_clip=llr_clip)
        gp, gm = g64.copy(), g64.copy()
        gp[j] += hh
        gm[j] -= hh
        fp, fm = lam64(gp), lam64(gm)
        cen, fwd, bwd = (fp - fm) / (2 * hh), (fp - f0) / hh, (f0 - fm) / hh
        smooth = (np.abs(fwd - bwd) <= 1e-5 * np.maximum(np.abs(cen), 1.0)) & agree[:, None]
        err = np.abs(dl - cen) / np.maximum(np.abs(cen), 1.0)
        assert err[smooth].max() < 1e-4, (j, err[smooth].max())
        checked += int((smooth & (np.abs(cen) > 1.0)).sum())
    assert checked > 1000, checked
    if llr_clip < 1e6:  # the clip is active: it changes the trajectory
        assert not np.array_equal(f0, oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, g64,
                                                   t_iters, syn, precision="f64")[:, t_iters])
