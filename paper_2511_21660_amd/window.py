"""Windowed Relay decoding over detector rounds (the overlapping windows of
T_commit + T_overlap rounds that the caveat of the paper's Sec. 7.3 describes:
decode a window, commit the faults of its first T_commit rounds, advance by
T_commit).

Reading of the windows (the paper gives only their outline): the matrix's
rows are detectors grouped in rounds of `band` rows and its columns are
sorted by the round of their first detector.  Window k covers detector
rounds [k*Tc, min(k*Tc + Tc + To, R)); its decoding problem holds the faults
whose first detector lies in those rounds, restricted to the window's rows,
and takes as syndrome the window's rows of the residual syndrome
sigma XOR H F_committed.  It commits the faults whose first detector lies in
its first Tc rounds (the last window, the one reaching round R, commits all
of its faults).  Every fault is committed by exactly one window.

Each window is an ordinary Relay decode on the GPU (rb_decode with the
window's own context); the residual syndrome is computed by rb_syndrome on
the full matrix's context.  This module only slices and copies device
buffers between those calls.
"""
from __future__ import annotations

import numpy as np

from . import relaybp


def window_plan(m, band, first_round, t_commit, t_overlap):
    """Windows as (row0, row1, col0, col1, col_commit): rows [row0, row1) and
    columns [col0, col1) of the window's problem, of which [col0, col_commit)
    are committed.  first_round must be non-decreasing (columns sorted)."""
    if t_commit < 1 or t_overlap < 0:
        raise ValueError("t_commit must be >= 1 and t_overlap >= 0")
    if band < 1 or m < 1:
        raise ValueError("m and band must be >= 1")
    first_round = np.asarray(first_round)
    if np.any(np.diff(first_round) < 0):
        raise ValueError("columns must be sorted by the round of their first detector")
    rounds = -(-m // band)
    plan = []
    s = 0
    while s < rounds:
        e = min(s + t_commit + t_overlap, rounds)
        last = e == rounds
        c0 = int(np.searchsorted(first_round, s, side="left"))
        c1 = int(np.searchsorted(first_round, e, side="left"))
        cc = c1 if last else int(np.searchsorted(first_round, s + t_commit, side="left"))
        plan.append((s * band, min(e * band, m), c0, c1, cc))
        if last:
            break
        s += t_commit
    return plan


class WindowedDecoder:
    """Relay decoding of a round-structured matrix in overlapping windows."""

    def __init__(self, problem, first_round, band, t_commit, t_overlap, device=0, **params):
        self.m, self.n = problem.m, problem.n
        if np.asarray(first_round).shape != (problem.n,):
            raise ValueError("first_round needs one entry per column")
        self.plan = window_plan(problem.m, band, first_round, t_commit, t_overlap)
        self.full = relaybp.Decoder.from_problem(problem, device=device, **params)
        self.decs = []
        rows, cols = np.asarray(problem.rows), np.asarray(problem.cols)
        for r0, r1, c0, c1, _ in self.plan:
            keep = (rows >= r0) & (rows < r1) & (cols >= c0) & (cols < c1)
            self.decs.append(relaybp.Decoder(r1 - r0, c1 - c0, rows[keep] - r0, cols[keep] - c0,
                                             problem.prior[c0:c1], device=device, **params))

    def close(self):
        for d in self.decs:
            d.close()
        self.full.close()

    def decode(self, syndromes, events=None):
        """syndromes: uint8 CUDA tensor [B, M].  Returns corr [B, N] (the
        committed faults of every window) and, per window, conv and iters
        ([W, B]) as CUDA tensors.  events (optional): one (start, end) pair of
        torch CUDA events per window, recorded around its decode on the
        current stream."""
        import torch

        if syndromes.dtype != torch.uint8 or syndromes.dim() != 2 or syndromes.shape[1] != self.m:
            raise ValueError(f"syndromes must be uint8 [B, {self.m}]")
        b = syndromes.shape[0]
        dev = syndromes.device
        syndromes = syndromes.contiguous()
        corr = torch.zeros((b, self.n), dtype=torch.uint8, device=dev)
        conv = torch.empty((len(self.plan), b), dtype=torch.uint8, device=dev)
        iters = torch.empty((len(self.plan), b), dtype=torch.int32, device=dev)
        residual = syndromes
        for k, ((r0, r1, c0, c1, cc), dec) in enumerate(zip(self.plan, self.decs)):
            win = residual[:, r0:r1].contiguous()
            if events is not None:
                events[k][0].record()
            out = dec.decode(win, want_weight=False)
            if events is not None:
                events[k][1].record()
            corr[:, c0:cc] = out["corr"][:, :cc - c0]
            conv[k] = out["conv"]
            iters[k] = out["iters"]
            if k + 1 < len(self.plan):
                residual = self.full.syndrome(corr, syn_in=syndromes)
        return {"corr": corr, "conv": conv, "iters": iters}
