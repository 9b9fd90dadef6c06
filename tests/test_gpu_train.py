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


def test_adjoint_deterministic_and_checkpoint_invariant(rb):
    prob, faults, syn, gamma = _setup(b=64, seed=5)
    runs = [_gpu_forward_backward(rb, prob, faults, syn, gamma, 1.0, 30, c) for c in (10, 10, 7, 30)]
    for r in runs[1:]:
        np.testing.assert_array_equal(runs[0][1], r[1])
        assert runs[0][2] == r[2]
