"""Learning Relay's leg-1 memory strengths through the unrolled decoder.

``RelayUnroll`` is a torch.autograd.Function around the library's
differentiable forward (rb_forward_train: T iterations of one DMem-BP leg with
per-column memory strengths gamma_j and channel LLRs s * w_j, checkpointed
every C iterations) and its hand-written adjoint (rb_backward).  Both passes
run in the HIP kernels; torch holds the tensors and the loss.

``soft_decoding_loss`` is the training objective: with q_j = P(F_j = 1) =
sigmoid(-Lambda_j(T)), a soft syndrome bit per check, P_i = (1 - prod_{j in
N(i)} (1 - 2 q_j)) / 2, scored by binary cross-entropy against sigma_i, plus a
soft logical bit per row a of the logical matrix, P_a = (1 - prod_{j in a}
(1 - 2 r_j)) / 2 with r_j = q_j if F_j = 0 else 1 - q_j (the probability that
the correction differs from the true faults at j), scored against 0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import relaybp


class RelayUnroll(torch.autograd.Function):
    """Lambda(T) [B, N] as a differentiable function of gamma [N] and scale [1]."""

    @staticmethod
    def forward(ctx, decoder, syndromes, gamma, scale, t_iters, ckpt_every):
        syndromes = syndromes.contiguous()
        gamma = gamma.detach().contiguous()
        scale = scale.detach().contiguous()
        b = syndromes.shape[0]
        tape = torch.empty(max(1, decoder.tape_bytes(b, t_iters, ckpt_every)), dtype=torch.uint8,
                           device=syndromes.device)
        llr = torch.empty((b, decoder.n), dtype=torch.float32, device=syndromes.device)
        decoder.forward_train(syndromes, gamma, scale, t_iters, ckpt_every, tape, llr)
        ctx.decoder, ctx.t_iters, ctx.ckpt_every = decoder, t_iters, ckpt_every
        ctx.save_for_backward(syndromes, gamma, scale, tape)
        return llr

    @staticmethod
    def backward(ctx, dllr):
        syndromes, gamma, scale, tape = ctx.saved_tensors
        dgamma = torch.empty_like(gamma)
        dscale = torch.empty_like(scale)
        ctx.decoder.backward_train(syndromes, gamma, scale, ctx.t_iters, ctx.ckpt_every, tape,
                                   dllr.contiguous().float(), dgamma, dscale)
        return None, None, dgamma, dscale, None, None


def incidence(rows, cols, m, n, device):
    h = torch.zeros((m, n), dtype=torch.float32, device=device)
    h[torch.as_tensor(rows, dtype=torch.long), torch.as_tensor(cols, dtype=torch.long)] = 1.0
    return h


def _odd_probability(log_abs, neg_count):
    """(1 - prod x)/2 from log|x| sums and the number of negative factors."""
    prod = torch.exp(log_abs) * (1.0 - 2.0 * torch.remainder(neg_count, 2.0))
    return 0.5 * (1.0 - prod)


def soft_decoding_loss(llr, syndromes, faults, h, logical, eps=1e-7):
    """Mean soft-syndrome BCE + mean soft-logical BCE (see module docstring).

    llr [B, N] float32, syndromes [B, M] uint8, faults [B, N] uint8, h [M, N] and
    logical [K, N] float 0/1 incidence matrices.
    """
    x = torch.tanh(0.5 * llr.double())  # 1 - 2 q_j
    ax = torch.clamp(x.abs(), min=1e-300).log()
    negx = (x < 0).double()
    p_syn = _odd_probability(ax @ h.double().T, negx @ h.double().T)
    s = syndromes.double()
    p_syn = p_syn.clamp(eps, 1 - eps)
    bce_syn = -(s * torch.log(p_syn) + (1 - s) * torch.log(1 - p_syn))
    f = faults.double()
    y = x * (1.0 - 2.0 * f)  # 1 - 2 r_j
    ay = torch.clamp(y.abs(), min=1e-300).log()
    negy = (y < 0).double()
    p_log = _odd_probability(ay @ logical.double().T, negy @ logical.double().T).clamp(eps, 1 - eps)
    bce_log = -torch.log(1 - p_log)
    return bce_syn.mean() + bce_log.mean()


def soft_decoding_loss_np(llr, syndromes, faults, h, logical, eps=1e-7):
    """The same loss in float64 numpy (for finite differences against the oracle)."""
    x = np.tanh(0.5 * np.asarray(llr, np.float64))
    hp = h.astype(np.float64)
    lp = logical.astype(np.float64)
    ax = np.log(np.maximum(np.abs(x), 1e-300))
    negx = (x < 0).astype(np.float64)
    prod = np.exp(ax @ hp.T) * (1.0 - 2.0 * np.mod(negx @ hp.T, 2.0))
    p_syn = np.clip(0.5 * (1.0 - prod), eps, 1 - eps)
    s = syndromes.astype(np.float64)
    bce_syn = -(s * np.log(p_syn) + (1 - s) * np.log(1 - p_syn))
    y = x * (1.0 - 2.0 * faults.astype(np.float64))
    ay = np.log(np.maximum(np.abs(y), 1e-300))
    negy = (y < 0).astype(np.float64)
    prod = np.exp(ay @ lp.T) * (1.0 - 2.0 * np.mod(negy @ lp.T, 2.0))
    p_log = np.clip(0.5 * (1.0 - prod), eps, 1 - eps)
    return bce_syn.mean() + (-np.log(1 - p_log)).mean()


def train_first_leg(decoder, problem, sample, steps=2000, t_iters=60, ckpt_every=10, lr=1e-2,
                    gamma_init=0.125, scale_init=1.0, log_every=100, log=None, gamma_range=None,
                    learn_scale=True):
    """Adam on (gamma_j, s) through the unrolled first leg.

    decoder: a relaybp.Decoder for `problem`; sample(step) -> (faults, syndromes)
    uint8 numpy arrays [B, N], [B, M] of freshly drawn errors.  t_iters: the
    unrolled depth, or a tuple of depths whose losses are averaged (each depth
    is one forward / adjoint pass from the initial LLRs).  gamma_range (lo, hi):
    learn gamma_j = lo + (hi - lo) sigmoid(theta_j) instead of gamma_j itself,
    which keeps every strength inside the range the paper draws later legs
    from (the adjoint gives dLoss/dgamma; torch applies the chain rule through
    the sigmoid).  learn_scale=False holds s at scale_init.  Returns (gamma
    float32 [N], scale float, history list of (step, loss)).
    """
    depths = (t_iters,) if isinstance(t_iters, int) else tuple(t_iters)
    dev = torch.device("cuda", decoder.device)
    if gamma_range is None:
        theta = torch.full((problem.n,), gamma_init, dtype=torch.float32, device=dev, requires_grad=True)

        def gamma_of(th):
            return th
    else:
        lo, hi = (float(x) for x in gamma_range)
        u0 = (gamma_init - lo) / (hi - lo)
        theta = torch.full((problem.n,), float(np.log(u0 / (1.0 - u0))), dtype=torch.float32, device=dev,
                           requires_grad=True)

        def gamma_of(th):
            return lo + (hi - lo) * torch.sigmoid(th)
    scale = torch.tensor([scale_init], dtype=torch.float32, device=dev, requires_grad=learn_scale)
    opt = torch.optim.Adam([theta, scale] if learn_scale else [theta], lr=lr)
    h = incidence(problem.rows, problem.cols, problem.m, problem.n, dev)
    lg = torch.from_numpy(problem.logical.astype(np.float32)).to(dev)
    history = []
    for step in range(steps):
        f, s = sample(step)
        d_syn = torch.from_numpy(s).to(dev)
        d_f = torch.from_numpy(f).to(dev)
        loss = 0.0
        gamma = gamma_of(theta)
        for t in depths:
            llr = RelayUnroll.apply(decoder, d_syn, gamma, scale, t, ckpt_every)
            loss = loss + soft_decoding_loss(llr, d_syn, d_f, h, lg)
        loss = loss / len(depths)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        if step % log_every == 0 or step == steps - 1:
            history.append((step, float(loss.item())))
            if log is not None:
                log(f"step {step} loss {history[-1][1]:.5f} scale {float(scale.item()):.4f}")
    return gamma_of(theta).detach().cpu().numpy(), float(scale.item()), history
