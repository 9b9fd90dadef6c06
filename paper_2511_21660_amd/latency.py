"""Latency-tail analysis of Relay decoding (paper Sec. 2.2: latency-tail
conditions and their slowdown bound; Sec. 7.2: real-time decoding despite
latency tails).

Decoding time is counted in iterations; the paper's FPGA design spends two
cycles per iteration (appendix on Relay resources), so FPGA cycles = 2 x
iterations.  Inputs are the per-shot outputs of one GPU decode:

* ``iters``  -- total iterations executed per shot (rb_decode's iters);
* ``failed`` -- per-shot logical failure (not converged, or the residual
  error F + F_hat acts on a logical).

With a single solution (S = 1) a decode stops at its first convergence, so a
run with an iteration budget T (``max_total_iters``) returns the same result
as the unbounded run for every shot with iters <= T and gives up (a failure)
on every other shot.  ``ler_vs_budget`` uses exactly that: one unbounded run
gives the logical error rate at every budget.
"""
from __future__ import annotations

import math

import numpy as np

CYCLES_PER_ITERATION = 2  # FPGA cycles per iteration in the paper's design


def finished_fraction(iters, budgets):
    """Fraction of shots whose decode ended within each budget (iterations)."""
    it = np.sort(np.asarray(iters, np.int64))
    return np.searchsorted(it, np.asarray(budgets, np.int64), side="right") / max(1, it.size)


def epsilon(iters, t_ref):
    """Probability that a decode runs longer than t_ref iterations."""
    it = np.asarray(iters, np.int64)
    return float(np.count_nonzero(it > t_ref)) / max(1, it.size)


def ler_vs_budget(iters, failed, budgets):
    """Logical error rate at each iteration budget T (single-solution decodes):
    P(failed and iters <= T) + P(iters > T)."""
    it = np.asarray(iters, np.int64)
    f = np.asarray(failed, bool)
    n = max(1, it.size)
    out = []
    for t in np.asarray(budgets, np.int64):
        out.append((np.count_nonzero(f & (it <= t)) + np.count_nonzero(it > t)) / n)
    return np.asarray(out)


def tail_factor(t_max, t_ref, t_gen):
    """ceil((T_max - T_ref) / (T_gen - T_ref)): how many generation periods a
    slow decode can overrun (requires T_ref < T_gen)."""
    if not t_ref < t_gen:
        raise ValueError("T_ref must be below T_gen")
    return math.ceil((t_max - t_ref) / (t_gen - t_ref))


def tail_gamma(eps, blocks, t_max, t_ref, t_gen):
    """gamma = eps * C * ceil((T_max - T_ref) / (T_gen - T_ref))."""
    return eps * blocks * tail_factor(t_max, t_ref, t_gen)


def tail_condition_holds(eps, blocks, t_max, t_ref, t_gen):
    """Both latency-tail conditions: T_ref / T_gen < 1 and gamma < 1."""
    return t_ref < t_gen and tail_gamma(eps, blocks, t_max, t_ref, t_gen) < 1.0


def max_blocks(eps, t_max, t_ref, t_gen):
    """Largest number of code blocks C for which gamma < 1 (inf if eps = 0)."""
    k = eps * tail_factor(t_max, t_ref, t_gen)
    if k <= 0:
        return math.inf
    c = math.ceil(1.0 / k) - 1
    return max(c, 0)


def slowdown_bound(eps, blocks, t_max, t_ref, t_gen, first_order=False):
    """Bound on the mean relative slowdown <R> < 1 + T_ref/T_gen + 2 gamma / (1 - gamma)
    (or its first-order form 1 + T_ref/T_gen + 2 gamma); requires gamma < 1."""
    g = tail_gamma(eps, blocks, t_max, t_ref, t_gen)
    if not g < 1.0:
        raise ValueError("latency-tail condition violated (gamma >= 1)")
    return 1.0 + t_ref / t_gen + (2.0 * g if first_order else 2.0 * g / (1.0 - g))


def summary(iters, failed, budgets_cycles, t_ref_cycles=500, t_gen_cycles=1000, blocks=10):
    """Dictionary of the analysis in FPGA cycles (2 per iteration): finished
    fraction and LER at each budget, epsilon(T_ref), and, taking each budget
    as T_max, the largest C meeting the tail condition and the slowdown bound
    for `blocks` code blocks."""
    b_it = [c // CYCLES_PER_ITERATION for c in budgets_cycles]
    t_ref_it = t_ref_cycles // CYCLES_PER_ITERATION
    eps = epsilon(iters, t_ref_it)
    fin = finished_fraction(iters, b_it)
    ler = ler_vs_budget(iters, failed, b_it)
    rows = []
    for c, f, l in zip(budgets_cycles, fin, ler):
        row = {"budget_cycles": int(c), "finished": float(f), "ler": float(l)}
        if c > t_ref_cycles:
            mb = max_blocks(eps, c, t_ref_cycles, t_gen_cycles)
            row["max_blocks"] = None if mb == math.inf else mb  # None: no tail observed
            if tail_condition_holds(eps, blocks, c, t_ref_cycles, t_gen_cycles):
                row["slowdown_bound"] = slowdown_bound(eps, blocks, c, t_ref_cycles, t_gen_cycles)
        rows.append(row)
    it = np.asarray(iters, np.int64)
    return {"t_ref_cycles": t_ref_cycles, "t_gen_cycles": t_gen_cycles, "blocks": blocks,
            "epsilon": eps, "max_cycles": int(it.max(initial=0)) * CYCLES_PER_ITERATION,
            "mean_cycles": float(it.mean()) * CYCLES_PER_ITERATION if it.size else 0.0,
            "budgets": rows}
