"""GPU tests of the differentiable decoder (learned memory strengths): forward
parity with the oracle, the hand-written adjoint against FP64 central finite
differences of the oracle, determinism and checkpoint invariance."""
import numpy as np
import pytest

import oracle
from tests.conftest import RELAY_DEFAULT
from workloads import codes, sampling

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2511_21660_amd import relaybp

    relaybp.load_library()
    return relaybp


def _setup(b=6, seed=3, p=0.04, name="bb144"):
    prob = codes.bb_problem(name, p)
    faults, syn = sampling.sample_batch(prob, (5 << 32) | seed, 0, b)
    rng = np.random.default_rng(seed)
    gamma = rng.uniform(0.0, 0.5, prob.n).astype(np.float32)
    return prob, faults, syn, gamma


def _gpu_forward_backward(rb, prob, faults, syn, gamma, scale, T, C):
    from paper_2511_21660_amd import learn

    dec = rb.Decoder.from_problem(prob, **RELAY_DEFAULT)
    d_syn = torch.from_numpy(syn).cuda()
    g = torch.tensor(gamma, device="cuda", requires_grad=True)
    s = torch.tensor([scale], dtype=torch.float32, device="cuda", requires_grad=True)
    llr = learn.RelayUnroll.apply(dec, d_syn, g, s, T, C)
    h = learn.incidence(prob.rows, prob.cols, prob.m, prob.n, "cuda")
    lg = torch.from_numpy(prob.logical.astype(np.float32)).cuda()
    loss = learn.soft_decoding_loss(llr, d_syn, torch.from_numpy(faults).cuda(), h, lg)
    loss.backward()
    torch.cuda.synchronize()
    return llr.detach().cpu().numpy(), g.grad.cpu().numpy(), float(s.grad.item()), float(loss)


def test_train_forward_equals_oracle_trace(rb):
    prob, faults, syn, gamma = _setup(b=8)
    for T, C, scale in ((60, 10, 1.0), (23, 7, 0.85)):
        llr, _, _, _ = _gpu_forward_backward(rb, prob, faults, syn, gamma, scale, T, C)
        ref = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, T, syn,
                           scale=scale)[:, T]
        np.testing.assert_array_equal(llr, ref)


def test_adjoint_matches_fp64_finite_differences(rb):
    """Central differences of the FP64 oracle loss (h = 1e-6) against the GPU
    adjoint, rel. tol. 1e-3, on coordinates with |g| > 1e-3 max|g| whose
    one-sided differences agree (no argmin / sign switch inside [x-h, x+h])."""
    from paper_2511_21660_amd import learn

    prob, faults, syn, gamma = _setup(b=4, seed=11)
    T, C, scale = 12, 5, 0.9
    _, g_gpu, s_gpu, _ = _gpu_forward_backward(rb, prob, faults, syn, gamma, scale, T, C)
    h_mat = prob.dense()

    def loss64(gam, sc):
        lam = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior,
                           gam.astype(np.float64), T, syn, scale=sc, precision="f64")[:, T]
        return learn.soft_decoding_loss_np(lam, syn, faults, h_mat, prob.logical)

    g64 = gamma.astype(np.float64)
    hh = 1e-6
    f0 = loss64(g64, scale)
    big = np.abs(g_gpu) > 1e-3 * np.abs(g_gpu).max()
    cand = np.nonzero(big)[0][:40]
    checked = 0
    for j in cand:
        gp, gm = g64.copy(), g64.copy()
        gp[j] += hh
        gm[j] -= hh
        fp, fm = loss64(gp, scale), loss64(gm, scale)
        fwd, bwd, cen = (fp - f0) / hh, (f0 - fm) / hh, (fp - fm) / (2 * hh)
        if abs(fwd - bwd) > 1e-4 * max(abs(cen), 1e-12):
            continue  # a kink inside the stencil: not differentiable there
        assert abs(g_gpu[j] - cen) <= 1e-3 * abs(cen), (j, g_gpu[j], cen)
        checked += 1
    assert checked >= 10
    fp, fm = loss64(g64, scale + hh), loss64(g64, scale - hh)
    cen = (fp - fm) / (2 * hh)
    assert abs(s_gpu - cen) <= 1e-3 * abs(cen), (s_gpu, cen)


def _setup_range(b, seed, lo, hi, p=0.04, name="bb144"):
    prob = codes.bb_problem(name, p)
    faults, syn = sampling.sample_batch(prob, (5 << 32) | seed, 0, b)
    gamma = np.random.default_rng(seed).uniform(lo, hi, prob.n).astype(np.float32)
    return prob, faults, syn, gamma


def test_adjoint_at_full_depth_matches_oracle_tangents(rb):
    """The adjoint at the training depth: T = 60 unrolled iterations with
    checkpoints every 10, 64 shots of [[144,12,12]] at p = 0.04, gamma_j drawn
    around the first-leg value (U(0.05, 0.2)).  Finite differences carry no
    information at this depth (Lambda grows to ~1e19 and the loss has a kink
    within 1e-10 of almost every point), so the reference is the oracle's
    forward-mode tangent along the same FP32 trajectory: for 40 coordinates
    with the largest |g_j|, g_j must equal sum_b <dL/dLambda_b(T),
    dLambda_b(T)/dgamma_j> with dL/dLambda in FP64, rel. tol. 1e-3; the scale
    to within the FP32 bound of its (ill-conditioned) sum."""
    from paper_2511_21660_amd import learn

    prob, faults, syn, gamma = _setup_range(64, 13, 0.05, 0.2)
    T, C, scale = 60, 10, 1.0
    llr, g_gpu, s_gpu, _ = _gpu_forward_backward(rb, prob, faults, syn, gamma, scale, T, C)
    ref = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, T, syn, scale=scale)[:, T]
    np.testing.assert_array_equal(llr, ref)
    lam = torch.from_numpy(llr.astype(np.float64)).requires_grad_(True)
    h = learn.incidence(prob.rows, prob.cols, prob.m, prob.n, "cpu")
    lg = torch.from_numpy(prob.logical.astype(np.float32))
    loss = learn.soft_decoding_loss(lam, torch.from_numpy(syn), torch.from_numpy(faults), h, lg)
    loss.backward()
    dl = lam.grad.numpy()
    assert np.abs(g_gpu).max() > 0.0
    order = np.argsort(-np.abs(g_gpu))[:40]
    for j in order:
        d = np.zeros(prob.n)
        d[j] = 1.0
        _, tan = oracle.tangent(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, T, syn, d, 0.0,
                                scale=scale)
        expect = float((dl * tan).sum())
        assert abs(g_gpu[j] - expect) <= 1e-3 * abs(expect), (j, g_gpu[j], expect)
    # The scale: dL/ds = sum_k d0_k w_k with d0_k = dL/dw'_k.  At this depth the
    # sum cancels to ~1e-8 of sum_k |d0_k w_k| (the shots that carry the loss
    # are chaotic), so FP32 can hold it only to eps32 * kappa; check the
    # oracle's two routes agree, and the GPU to within that bound.
    w = np.log((1.0 - prob.prior) / prob.prior).astype(np.float32).astype(np.float64)
    d0 = np.zeros(prob.n)
    for k in range(prob.n):
        d = np.zeros(prob.n)
        d[k] = 1.0
        _, tan = oracle.tangent(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, T, syn,
                                np.zeros(prob.n), 0.0, scale=scale, dwprime=d)
        d0[k] = float((dl * tan).sum())
    _, tan = oracle.tangent(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, T, syn,
                            np.zeros(prob.n), 1.0, scale=scale)
    expect = float((dl * tan).sum())
    kappa = float(np.abs(d0 * w).sum())
    assert abs(expect - float((d0 * w).sum())) <= 1e-9 * kappa
    assert abs(s_gpu - expect) <= 1e-3 * abs(expect) + 2.0 ** -23 * kappa, (s_gpu, expect, kappa)


def test_adjoint_deterministic_and_checkpoint_invariant(rb):
    prob, faults, syn, gamma = _setup(b=64, seed=5)
    runs = [_gpu_forward_backward(rb, prob, faults, syn, gamma, 1.0, 30, c) for c in (10, 10, 7, 30)]
    for r in runs[1:]:
        np.testing.assert_array_equal(runs[0][1], r[1])
        assert runs[0][2] == r[2]
