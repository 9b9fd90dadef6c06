#!/usr/bin/env python3
"""Relay-BP decoding throughput on one MI355X.

Default workload (--workload dem, the headline): plain Relay-BP FP32 on the
DEM-shaped synthetic 936 x 8785 matrix (13 rounds of 72 detectors, columns of
weight 2-6, E = 27,617 edges, priors log-uniform in [1e-4, 1e-2]), 10^6
syndromes per step already resident in HBM, T_1 = 80, T_r = 60, R = 20 legs,
S = 1, memory strengths gamma_1 = 0.125 and U[-0.24, 0.66] after; syndromes
in and corrections out bit-packed in uint32 words (--io-layout bytes: one
byte per entry).  With the latency tail: completion and LER within FPGA-cycle budgets, epsilon(T_ref)
and the latency-tail condition.

Other workloads:
  --workload bb144        [[144,12,12]] code capacity, p in {0.02, 0.04, 0.06, 0.08},
                          10^5 syndromes per p in one launch, R = 301, S = 5
  --workload dem-2gross   two-gross-scale DEM-shaped 2736 x 26208 matrix (82.6K edges)
                          on the large-graph kernel, 2 x 10^5 shots, R = 20, S = 1
  --workload dem-window   the DEM-shaped matrix decoded in overlapping windows of
                          T_commit = T_overlap = 3 detector rounds (4 windows), 2 x 10^5
                          shots, R = 20, S = 1; LER against the full-matrix decode
  --workload bp-llr       plain min-sum BP (one leg, gamma = 0, 25 rounds) on the
                          DEM-shaped matrix, 10^5 shots, returning the marginals
  --workload mixed-codes  [[72,12,6]], [[90,8,10]], [[144,12,12]], [[288,12,18]]
                          interleaved 4:3:2:1, 4 x 10^5 shots at p = 0.04, R = 20,
                          S = 1: one autotuned mixed launch (eager and replayed from
                          a hipGraph) against four per-code launches
  --workload learned      [[144,12,12]] at p = 0.04: learn gamma_j and the prior
                          scale through 60 unrolled iterations (2000 Adam steps,
                          batch 4096; lr 1e-2 with the loss at T = 60, free and with
                          gamma_j = lo + (hi - lo) sigmoid(theta_j) in the paper's
                          range, that with the scale held at 1, and lr 1e-3 with
                          the loss averaged over T = 5..60),
                          then decode 10^6 held-out shots with Relay (R = 20, S = 1)
                          and one DMem-BP leg (T = 60), with and without the learned
                          first leg

Prints one JSON line: syndromes/s (the headline), edge-updates/s, the ALU
roofline of the decode kernel from HIP events on the launch stream, the LDS
roofline, the logical error rate with 95 % Wilson intervals, and the CPU
oracle timed on a bounded sample of the same syndromes on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks (published): 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 39.3 T lane-ops/s (non-packed FP32 / int)
# LDS read bandwidth of gfx950, measured by paper_2511_21660_amd/ldspeak.py:
# conflict-free ds_read_b128 and _b64 reach 234 and 228 B/clk/CU, so the peak
# is taken as 256 B/clk/CU (CDNA3's 128 B/clk is half of it); ds_read_b32
# reaches 117 of its 128 B/clk (256 bytes per wave every two clocks), the
# ceiling for the 4-byte gathers the decoders issue.
PEAK_LDS_TBS = 256 * 256 * 2.4e9 / 1e12       # 157.3 TB/s at 256 B/clk/CU
PEAK_LDS_B32_TBS = 256 * 128 * 2.4e9 / 1e12   # 78.6 TB/s for 4-byte reads

# Relay parameters of the paper's appendix on Relay resources (T = 80, then
# 60; gamma_0 = 0.125, gamma ~ U[-0.24, 0.66]); R counts every leg.
RELAY = dict(num_legs=301, iters_first=80, iters_leg=60, num_solutions=5, gamma_first=0.125,
             gamma_lo=-0.24, gamma_hi=0.66, llr_clip=2.0 ** 64, seed=0x52454C4159, anchor=0,
             max_total_iters=0)
RELAY_R20 = dict(RELAY, num_legs=20, num_solutions=1)

# Algorithmic work per edge-update (one edge in one iteration), from the
# update rules: check side nu = clip(Lambda - mu) (2), sign parity (1), the
# two smallest magnitudes and the position of the smallest (compare, min1,
# min2, position: 4), per-edge magnitude select (2) and sign (1); fault side
# sum (1); syndrome parity (1) => 12 per edge, plus per fault 7 (1 - gamma,
# two products, sum, two clips, decision) and per check 3.
OPS_PER_EDGE = 12.0
OPS_PER_FAULT = 7.0
OPS_PER_CHECK = 3.0

DEFAULT_STEPS = {"bb144": 20, "dem": 5, "dem-2gross": 3, "dem-window": 3, "mixed-codes": 10, "learned": 3,
                 "bp-llr": 10}


def ops_per_iteration(m, n, e):
    return OPS_PER_EDGE * e + OPS_PER_FAULT * n + OPS_PER_CHECK * m


def lds_bytes_per_edge_update(m, n, e):
    """Algorithmic LDS bytes per edge-update: one nu to its check and one mu
    back (8 B), plus Lambda / lambda per fault (8 B) and the check state
    (12 B) per check, spread over the edges."""
    return 8.0 + (8.0 * n + 12.0 * m) / e


def lds_bytes_per_edge_update_large(m, n, e, row_deg):
    """The same for the large-graph kernel's compressed messages: Lambda to
    the check (4 B) and one 16-byte check record (state and the edge's sign
    word) to the fault; a byte of nu signs read and written per 8 row
    positions; per check its state read (12 B) and written to each of its
    records (12 B, one record per 32 positions); per fault Lambda read and
    written."""
    row_deg = np.asarray(row_deg, dtype=np.int64)
    records = int(np.maximum(1, (row_deg + 31) // 32).sum())
    return 20.0 + 2.0 / 8.0 + (12.0 * m + 12.0 * records + 8.0 * n) / e


def wilson(k, n, z=1.96):
    if n == 0:
        return (0.0, 0.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def logical_failures(prob, faults, corr, conv):
    resid = (faults ^ corr).astype(np.int64)
    bad = ((prob.logical.astype(np.int64) @ resid.T) % 2).any(0)
    return (~conv.astype(bool)) | bad


WARM_SECONDS = 0.3  # the GPU's clocks ramp up over the first ~0.1-0.3 s of load


def timed(torch, step, n_launch, steps, warmup):
    """warmup untimed steps (continued, up to 1000 steps, until WARM_SECONDS
    have passed, so that short launches are not timed at idle clocks), then
    `steps` steps bracketed by device synchronisation.  step(ev) records ev[k]
    = (start, end) HIP events on the launch stream around launch k (ev is None
    during warm-up)."""
    t_warm = time.perf_counter()
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    extra = 0
    while time.perf_counter() - t_warm < WARM_SECONDS and extra < 1000:
        step(None)
        torch.cuda.synchronize()
        extra += 1
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n_launch)]
        step(ev)
        evs.append(ev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_launch = [[e[0].elapsed_time(e[1]) for e in ev] for ev in evs]
    return elapsed, per_launch


def launch_means(per_launch):
    return [float(np.mean([pl[k] for pl in per_launch])) for k in range(len(per_launch[0]))]


def roofline(kernel, kernel_ms, ops_launch, eu_launch, lds_b_per_eu, traffic):
    achieved = ops_launch / (kernel_ms * 1e-3) / 1e12
    lds = eu_launch * lds_b_per_eu / (kernel_ms * 1e-3) / 1e12
    return ({"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "Tops/s",
             "frac": achieved / PEAK_VALU_TOPS, "traffic": traffic, "kernel": kernel,
             "kernel_ms_per_launch": kernel_ms, "ops_per_edge_update": ops_launch / eu_launch},
            {"achieved": lds, "peak": PEAK_LDS_TBS, "unit": "TB/s", "frac": lds / PEAK_LDS_TBS,
             "frac_of_b32_read_peak": lds / PEAK_LDS_B32_TBS,
             "bytes_per_edge_update": lds_b_per_eu})


def stored_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 summary, if it was taken
    with the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    from paper_2511_21660_amd import profiling

    rec = json.load(open(path))
    if rec.get("source_hash") != profiling.source_hash():
        return None
    return rec["traffic_bytes_per_launch"]


def head(args, value, elapsed, config):
    return {
        "metric": "syndromes decoded/s at matched LER; edge-updates/s and % HBM/LDS roofline",
        "value": value,
        "unit": "syndromes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_note": f"each timed loop runs its warmup steps, then untimed steps until {WARM_SECONDS} s "
                       "of load have passed (clock ramp-up)",
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
    }


def oracle_threads():
    return min(16, len(os.sched_getaffinity(0)) or 1)


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def oracle_baseline(decode_sample, n_all, n_one, total, what):
    """Times the oracle on the first n_all syndromes with oracle_threads()
    threads and on the first n_one with one thread.  decode_sample(n, threads)
    runs the oracle and returns whether its outputs equal the GPU's."""
    threads = oracle_threads()
    t1 = time.perf_counter()
    agree = decode_sample(n_all, threads)
    tc = time.perf_counter() - t1
    t1 = time.perf_counter()
    agree1 = decode_sample(n_one, 1)
    t_one = time.perf_counter() - t1
    return {"value": n_all / tc, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_all} of {total} {what}, same inputs, {tc:.1f} s on {threads} threads; "
                      f"first {n_one} on one thread, {t_one:.1f} s",
            "one_core": {"value": n_one / t_one, "shots": n_one},
            "host": host_cpu(),
            "paired_with_gpu_bit_exact": bool(agree and agree1)}


# --------------------------------------------------------------------------
# [[144,12,12]] at four p values, S = 5
# --------------------------------------------------------------------------


def run_bb144(args, torch, rb, codes, sampling):
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    ps = [0.02, 0.04, 0.06, 0.08]
    shots = args.shots or 100000
    probs, faults, syns = [], [], []
    for q, p in enumerate(ps):
        prob = codes.bb_problem("bb144", p)
        f, s = sampling.sample_batch(prob, (2 << 32) | q, 0, shots)
        probs.append(prob)
        faults.append(f)
        syns.append(s)
    M, N, E = probs[0].m, probs[0].n, probs[0].nnz
    if args.schedule == "mixed":
        mdec = rb.MultiDecoder(probs, device=0, **RELAY)
        code_id = torch.cat([torch.full((s.shape[0],), q, dtype=torch.int32)
                             for q, s in enumerate(syns)]).to(dev)
        d_all = torch.from_numpy(np.concatenate(syns)).to(dev)
        mout = mdec.alloc(d_all.shape[0])
        offs = np.cumsum([0] + [s.shape[0] for s in syns])

        def step(ev):
            if ev is not None:
                ev[0][0].record(stream)
            mdec.decode(code_id, d_all, out=mout)
            if ev is not None:
                ev[0][1].record(stream)

        n_launch, kernel, info = 1, "relay_mixed_kernel", {"variant": "mixed"}

        def results():
            host = {k: v.cpu().numpy() for k, v in mout.items() if k != "workspace"}
            return [{k: v[offs[q]:offs[q + 1]] for k, v in host.items()} for q in range(len(ps))]
    else:
        decs = [rb.Decoder.from_problem(pr, device=0, **RELAY) for pr in probs]
        for d in decs:
            if args.variant is not None:
                d.set_variant(args.variant)
            if args.schedule == "per-p-lpt":
                d.reserve(shots)
        d_syn = [torch.from_numpy(s).to(dev) for s in syns]
        outs = [decs[q].decode(d_syn[q]) for q in range(len(ps))]

        def step(ev):
            for q in range(len(ps)):
                if ev is not None:
                    ev[q][0].record(stream)
                decs[q].decode(d_syn[q], out=outs[q])
                if ev is not None:
                    ev[q][1].record(stream)

        n_launch, kernel = len(ps), "relay_group_kernel"
        info = decs[0].info()

        def results():
            return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]

    elapsed, per_launch = timed(torch, step, n_launch, args.steps, args.warmup)
    kernel_ms = float(np.mean(per_launch))
    res = results()
    n_shots = sum(s.shape[0] for s in syns)
    iters_step = sum(int(r["iters"].astype(np.int64).sum()) for r in res)
    eu_launch = iters_step * E / n_launch
    traffic = stored_traffic("relay_mixed_kernel_bb144_hbm_traffic.txt") if n_launch == 1 else None
    roof, lds = roofline(kernel, kernel_ms, eu_launch / E * ops_per_iteration(M, N, E), eu_launch,
                         lds_bytes_per_edge_update(M, N, E), traffic)
    ler = {}
    for q, p in enumerate(ps):
        fail = logical_failures(probs[q], faults[q], res[q]["corr"][:, :N], res[q]["conv"])
        k = int(fail.sum())
        ler[str(p)] = {"ler": k / len(fail), "wilson95": wilson(k, len(fail)),
                       "conv": float(res[q]["conv"].mean()),
                       "mean_iters": float(res[q]["iters"].mean()),
                       "max_iters": int(res[q]["iters"].max())}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle_threads()
        n_cpu = min(args.cpu_sample or shots, shots)
        t1 = time.perf_counter()
        agree = True
        for q in range(len(ps)):
            ref = oracle.decode(probs[q].m, probs[q].n, probs[q].rows, probs[q].cols,
                                probs[q].prior, RELAY, syns[q][:n_cpu], threads=threads)
            agree &= bool(np.array_equal(ref["corr"], res[q]["corr"][:n_cpu, :N])
                          and np.array_equal(ref["iters"], res[q]["iters"][:n_cpu]))
        tc = time.perf_counter() - t1
        cpu = {"value": len(ps) * n_cpu / tc, "unit": "syndromes/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {n_cpu} syndromes of each of the 4 p values "
                         f"({len(ps) * n_cpu} of {n_shots}), same inputs, {tc:.1f} s",
               "paired_with_gpu_bit_exact": agree}
    f16 = None
    if args.f16_steps > 0:
        # the same syndromes with binary16 messages (block kernel, two syndromes
        # per workgroup): LER per p beside FP32's, and the bit-exact pairing
        # with the oracle's binary16 mode on the first 2000 syndromes of each p
        f16 = {}
        decs16 = [rb.Decoder.from_problem(pr, device=0, **dict(RELAY, precision=1)) for pr in probs]
        d16 = [torch.from_numpy(s).to(dev) for s in syns]
        outs16 = [decs16[q].decode(d16[q]) for q in range(len(ps))]

        def step16(ev):
            for q in range(len(ps)):
                if ev is not None:
                    ev[q][0].record(stream)
                decs16[q].decode(d16[q], out=outs16[q])
                if ev is not None:
                    ev[q][1].record(stream)

        el16, pl16 = timed(torch, step16, len(ps), args.f16_steps, 1)
        it16 = sum(int(o["iters"].to(torch.int64).sum().item()) for o in outs16)
        ms16 = float(np.sum(launch_means(pl16)))
        roof16 = {"bound": "alu", "achieved": it16 * ops_per_iteration(M, N, E) / (ms16 * 1e-3) / 1e12,
                  "peak": 2 * PEAK_VALU_TOPS, "unit": "Tops/s", "kernel": "relay_block16_kernel",
                  "peak_note": "packed binary16: two lane-ops per lane per cycle"}
        roof16["frac"] = roof16["achieved"] / roof16["peak"]
        f16["throughput"] = {"syndromes_per_s": n_shots * args.f16_steps / el16,
                             "kernel_ms_per_step": ms16, "roofline": roof16,
                             "note": "four per-p launches of the block kernel's binary16 form (two syndromes "
                                     "per workgroup); FP32 above runs the group kernel"}
        for q, p in enumerate(ps):
            dec16 = decs16[q]
            o = {k: v.cpu().numpy() for k, v in outs16[q].items()}
            fail = logical_failures(probs[q], faults[q], o["corr"], o["conv"])
            kf = int(fail.sum())
            ent = {"ler": kf / len(fail), "wilson95": wilson(kf, len(fail)), "mean_iters": float(o["iters"].mean()),
                   "same_correction_as_fp32": float((o["corr"] == res[q]["corr"][:, :N]).all(1).mean())}
            if not args.no_cpu_baseline:
                import oracle

                n = min(2000, len(fail))
                ref = oracle.decode(probs[q].m, probs[q].n, probs[q].rows, probs[q].cols, probs[q].prior, RELAY,
                                    syns[q][:n], precision="h16", threads=oracle_threads())
                ent["oracle_h16_paired_bit_exact"] = bool(np.array_equal(ref["corr"], o["corr"][:n])
                                                          and np.array_equal(ref["iters"], o["iters"][:n]))
            f16[str(p)] = ent
            dec16.close()
    line = head(args, n_shots * args.steps / elapsed, elapsed, {
        "workload": "relay_bp_bb144_code_capacity", "code": "[[144,12,12]] HX 72x144",
        "edges": E, "p": ps, "syndromes_per_p": shots, "syndromes_per_step": n_shots,
        "T_first": 80, "T_leg": 60, "legs": 301, "solutions": 5, "gamma_first": 0.125,
        "gamma_range": [-0.24, 0.66], "anchor": "chain", "schedule": args.schedule,
        "parallelism": "single_gpu"})
    line.update({"edge_updates_per_s": iters_step * E * args.steps / elapsed,
                 "launch_ms": launch_means(per_launch), "roofline": roof, "lds_roofline": lds,
                 "ler": ler, "binary16": f16, "kernel_config": info, "cpu_baseline": cpu})
    return line


# --------------------------------------------------------------------------
# DEM-shaped 936 x 8785 matrix, 10^6 shots, R = 20, S = 1
# --------------------------------------------------------------------------


def end_to_end(torch, dec, syn_np, out):
    """One decode with the copies: syndromes from pinned host memory to the
    device, the decode, and corrections, converged flags, legs and iterations
    back to pinned host memory, timed by the wall clock around synchronised
    copies (reported beside the HBM-resident rate, never as it)."""
    dev = out["corr"].device
    h_syn = torch.from_numpy(syn_np).pin_memory()
    h_out = {k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True)
             for k, v in out.items() if k in ("corr", "conv", "legs", "iters")}
    d_syn = torch.empty(h_syn.shape, dtype=h_syn.dtype, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d_syn.copy_(h_syn, non_blocking=True)
    dec.decode(d_syn, out=out)
    for k, v in h_out.items():
        v.copy_(out[k], non_blocking=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h2d = h_syn.numel() * h_syn.element_size()
    d2h = sum(v.numel() * v.element_size() for v in h_out.values())
    same = bool(torch.equal(h_out["corr"][:20000], out["corr"][:20000].cpu()))
    return {"syndromes_per_s": syn_np.shape[0] / el, "ms": el * 1e3, "h2d_bytes": h2d, "d2h_bytes": d2h,
            "first_20000_identical": same}


def measure_h16(args, torch, rb, prob, d_syn, syn_np, bits, failures, corr_bytes, out32, stream):
    """The same syndromes decoded with binary16 messages (two syndromes per
    workgroup): throughput, the packed-FP16 ALU roofline, LER with its Wilson
    interval beside FP32's, agreement with the FP32 decisions, and bit-exact
    pairing with the oracle's binary16 mode on a sample."""
    M, N, E = prob.m, prob.n, prob.nnz
    shots = syn_np.shape[0]
    dec = rb.Decoder.from_problem(prob, device=0, **dict(RELAY_R20, io_layout=1 if bits else 0, precision=1))
    o = dec.decode(d_syn)

    def step(ev):
        if ev is not None:
            ev[0][0].record(stream)
        dec.decode(d_syn, out=o)
        if ev is not None:
            ev[0][1].record(stream)

    elapsed, per_launch = timed(torch, step, 1, args.f16_steps, 1)
    kernel_ms = float(np.mean(per_launch))
    iters = o["iters"].cpu().numpy()
    it = int(iters.astype(np.int64).sum())
    achieved = it * ops_per_iteration(M, N, E) / (kernel_ms * 1e-3) / 1e12
    fail = failures(o)
    k = int(fail.sum().item())
    same = 0
    for s0 in range(0, shots, 50000):
        same += int((corr_bytes(s0, s0 + 50000, o) == corr_bytes(s0, s0 + 50000)).all(1).sum().item())
    res = {"syndromes_per_s": shots * args.f16_steps / elapsed, "launch_ms": kernel_ms,
           "roofline": {"bound": "alu", "achieved": achieved, "peak": 2 * PEAK_VALU_TOPS, "unit": "Tops/s",
                        "frac": achieved / (2 * PEAK_VALU_TOPS), "kernel": "relay_block16_kernel",
                        "peak_note": "packed binary16: two lane-ops per lane per cycle"},
           "lds_roofline": {"achieved": it * E * lds_bytes_per_edge_update(M, N, E) / 2 / (kernel_ms * 1e-3) / 1e12,
                            "peak": PEAK_LDS_TBS, "unit": "TB/s",
                            "note": "algorithmic bytes of binary16 messages: half of the FP32 figure"},
           "ler": k / shots, "wilson95": wilson(k, shots), "conv": float(o["conv"].float().mean().item()),
           "mean_iters": float(iters.mean()), "same_correction_as_fp32": same / shots,
           "clip": "min(L, 4096)", "steps": args.f16_steps}
    res["lds_roofline"]["frac"] = res["lds_roofline"]["achieved"] / PEAK_LDS_TBS
    if not args.no_cpu_baseline:
        import oracle

        n = min(1000, shots)
        t1 = time.perf_counter()
        ref = oracle.decode(M, N, prob.rows, prob.cols, prob.prior, RELAY_R20, syn_np[:n], precision="h16",
                            threads=oracle_threads())
        tc = time.perf_counter() - t1
        res["oracle_h16"] = {"shots": n, "syndromes_per_s": n / tc,
                             "paired_with_gpu_bit_exact": bool(
                                 np.array_equal(ref["corr"], corr_bytes(0, n, o).cpu().numpy())
                                 and np.array_equal(ref["iters"], iters[:n])
                                 and np.array_equal(ref["conv"], o["conv"][:n].cpu().numpy()))}
    dec.close()
    return res


def run_dem(args, torch, rb, codes, sampling, two_gross=False):
    """DEM-shaped matrix: 936 x 8785 on the block kernel, or (two_gross) the
    two-gross-scale 2736 x 26208 on the large-graph kernel."""
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    prob = codes.dem_problem(2736, 26208) if two_gross else codes.dem_problem()
    M, N, E = prob.m, prob.n, prob.nnz
    tag = f"{M}x{N}"
    shots = args.shots or (200000 if two_gross else 1000000)
    t_in = time.perf_counter()
    syn_np, (f_shots, f_cols) = sampling.sample_syndromes_sparse(prob, 0xDE3, shots)
    print(f"# dem {tag} inputs: {shots} shots, {f_shots.size} faults, "
          f"{time.perf_counter() - t_in:.1f} s", file=sys.stderr, flush=True)
    bits = args.io_layout == "bits32"
    dec = rb.Decoder.from_problem(prob, device=0, **dict(RELAY_R20, io_layout=1 if bits else 0))
    if args.variant is not None:
        dec.set_variant(args.variant)
    d_syn = torch.from_numpy(rb.pack_bits(syn_np) if bits else syn_np).to(dev)
    out = dec.decode(d_syn)

    def corr_bytes(s0, s1, o=None):
        """Corrections of shots s0 .. s1 - 1 (of `o`, default the FP32 decode) as
        uint8 [s1 - s0, N] on the device."""
        c = (out if o is None else o)["corr"][s0:s1]
        if not bits:
            return c
        sh = torch.arange(32, device=dev, dtype=torch.int32)
        return ((c[:, :, None] >> sh) & 1).reshape(c.shape[0], -1)[:, :N].to(torch.uint8)

    def step(ev):
        if ev is not None:
            ev[0][0].record(stream)
        dec.decode(d_syn, out=out)
        if ev is not None:
            ev[0][1].record(stream)

    elapsed, per_launch = timed(torch, step, 1, args.steps, args.warmup)
    kernel_ms = float(np.mean(per_launch))
    iters = out["iters"].cpu().numpy()
    conv = out["conv"].cpu().numpy()
    iters_launch = int(iters.astype(np.int64).sum())
    kernel = "relay_large_kernel" if two_gross else "relay_block_kernel"
    lds_b = (lds_bytes_per_edge_update_large(M, N, E, np.bincount(prob.rows, minlength=M)) if two_gross
             else lds_bytes_per_edge_update(M, N, E))
    roof, lds = roofline(kernel, kernel_ms, iters_launch * ops_per_iteration(M, N, E), iters_launch * E, lds_b,
                         stored_traffic(f"{kernel}_dem{tag}_hbm_traffic.txt"))
    # logical failures on the GPU, so that the correction array stays in HBM:
    # A (F xor F_hat) = A F xor A F_hat over GF(2).
    a = torch.from_numpy(prob.logical.astype(np.float32)).to(dev)
    af = torch.zeros((shots, a.shape[0]), dtype=torch.int32, device=dev)
    d_fs = torch.from_numpy(f_shots).to(dev)
    d_fc = torch.from_numpy(f_cols).to(dev)
    for c0 in range(0, d_fs.numel(), 1 << 22):
        af.index_add_(0, d_fs[c0:c0 + (1 << 22)],
                      a[:, d_fc[c0:c0 + (1 << 22)]].T.contiguous().to(torch.int32))
    def failures(o):
        bad = torch.zeros(shots, dtype=torch.bool, device=dev)
        for s0 in range(0, shots, 50000):
            ah = torch.round(corr_bytes(s0, s0 + 50000, o).float() @ a.T).to(torch.int32)
            bad[s0:s0 + 50000] = ((ah + af[s0:s0 + 50000]) % 2).any(1)
        return bad | (o["conv"] == 0)

    fail = failures(out)
    k = int(fail.sum().item())
    f16 = None
    if not two_gross and args.f16_steps > 0:
        f16 = measure_h16(args, torch, rb, prob, d_syn, syn_np, bits, failures, corr_bytes, out, stream)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        def decode_sample(n, threads):
            ref = oracle.decode(M, N, prob.rows, prob.cols, prob.prior, RELAY_R20, syn_np[:n],
                                threads=threads)
            return bool(np.array_equal(ref["corr"], corr_bytes(0, n).cpu().numpy())
                        and np.array_equal(ref["iters"], iters[:n])
                        and np.array_equal(ref["legs"], out["legs"][:n].cpu().numpy())
                        and np.array_equal(ref["conv"], conv[:n]))

        n_cpu = min(args.cpu_sample or (200 if two_gross else 20000), shots)
        cpu = oracle_baseline(decode_sample, n_cpu, max(1, n_cpu // (16 if two_gross else 40)), shots,
                              "syndromes")
    e2e = end_to_end(torch, dec, rb.pack_bits(syn_np) if bits else syn_np, out) if not two_gross else None
    line = head(args, shots * args.steps / elapsed, elapsed, {
        "workload": f"relay_bp_dem_{tag}", "matrix": f"DEM-shaped synthetic {tag}",
        "edges": E, "shots": shots, "T_first": 80, "T_leg": 60, "legs": 20, "solutions": 1,
        "gamma_first": 0.125, "gamma_range": [-0.24, 0.66], "anchor": "chain",
        "io_layout": args.io_layout, "parallelism": "single_gpu"})
    # latency tail (Sec. 7.2): completion within FPGA-cycle budgets (2 cycles
    # per iteration), LER at each budget, epsilon(T_ref = 500 cycles), and the
    # latency-tail condition for T_gen = 1000 cycles and C = 10 code blocks
    from paper_2511_21660_amd import latency

    tail = latency.summary(iters, fail.cpu().numpy(), [100, 200, 300, 500, 1000, 1500, 2440],
                           t_ref_cycles=500, t_gen_cycles=1000, blocks=10)
    line.update({"edge_updates_per_s": iters_launch * E * args.steps / elapsed,
                 "launch_ms": [kernel_ms], "roofline": roof, "lds_roofline": lds,
                 "ler": {"ler": k / shots, "wilson95": wilson(k, shots),
                         "conv": float(conv.mean()), "mean_iters": float(iters.mean()),
                         "max_iters": int(iters.max()), "faults_per_shot": f_shots.size / shots},
                 "latency_tail": tail, "kernel_config": dec.info(), "end_to_end": e2e,
                 "binary16": f16, "cpu_baseline": cpu})
    return line


# --------------------------------------------------------------------------
# windowed decoding of the DEM-shaped matrix (T_commit + T_overlap rounds)
# --------------------------------------------------------------------------


def run_dem_window(args, torch, rb, codes, sampling):
    """Windows of Tc = To = 3 detector rounds (72 detectors per round, 13
    rounds) over the DEM-shaped 936 x 8785 matrix: 4 window decodes per batch
    (block kernel) plus the residual-syndrome kernel between them."""
    from paper_2511_21660_amd import window

    dev = torch.device("cuda", 0)
    prob, first = codes.dem_rounds_problem()
    band, tc, to = 72, 3, 3
    shots = args.shots or 200000
    f_np, syn_np = sampling.sample_batch(prob, 0xDE4 << 32, 0, shots)
    wd = window.WindowedDecoder(prob, first, band, tc, to, device=0, **RELAY_R20)
    d_syn = torch.from_numpy(syn_np).to(dev)
    nw = len(wd.plan)
    holder = {}

    def step(ev):
        # HIP events on the launch stream around each window's decode
        holder["out"] = wd.decode(d_syn, events=ev)

    elapsed, per_launch = timed(torch, step, nw, args.steps, args.warmup)
    win_ms = launch_means(per_launch)
    out = holder["out"]
    iters = out["iters"].cpu().numpy().astype(np.int64)  # [W, B]
    conv = out["conv"].cpu().numpy()
    ops = 0.0
    eu = 0.0
    for k, (r0, r1, c0, c1, _) in enumerate(wd.plan):
        keep = (prob.rows >= r0) & (prob.rows < r1) & (prob.cols >= c0) & (prob.cols < c1)
        ew = int(keep.sum())
        ops += float(iters[k].sum()) * ops_per_iteration(r1 - r0, c1 - c0, ew)
        eu += float(iters[k].sum()) * ew
    kernel_ms = float(sum(win_ms))
    roof, lds = roofline("relay_block_kernel", kernel_ms, ops, eu, lds_bytes_per_edge_update(prob.m, prob.n, prob.nnz),
                         None)
    # logical failures on the GPU in chunks: A (F xor F_hat) over GF(2)
    a_t = torch.from_numpy(prob.logical.astype(np.float32)).to(dev)
    d_f = torch.from_numpy(f_np).to(dev)

    def failures(d_corr, d_ok):
        bad = torch.zeros(shots, dtype=torch.bool, device=dev)
        for s0 in range(0, shots, 50000):
            r = (d_f[s0:s0 + 50000] ^ d_corr[s0:s0 + 50000]).float()
            bad[s0:s0 + 50000] = (torch.round(r @ a_t.T).to(torch.int32) % 2).any(1)
        return (bad | ~d_ok.bool()).cpu().numpy()

    fail = failures(out["corr"], out["conv"].bool().all(0))
    k_fail = int(fail.sum())
    full = rb.Decoder.from_problem(prob, device=0, **RELAY_R20)
    fo = full.decode(d_syn)
    fail_full = failures(fo["corr"], fo["conv"].bool())
    full.close()
    corr = out["corr"][: min(shots, args.cpu_sample or 300)].cpu().numpy()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle_threads()
        n_cpu = min(args.cpu_sample or 300, shots)
        t1 = time.perf_counter()
        ref = oracle.decode_windowed(prob.m, prob.n, prob.rows, prob.cols, prob.prior, RELAY_R20, syn_np[:n_cpu],
                                     band, first, tc, to, threads=threads)
        tcpu = time.perf_counter() - t1
        agree = bool(np.array_equal(ref["corr"], corr[:n_cpu]) and np.array_equal(ref["iters"], iters[:, :n_cpu]))
        cpu = {"value": n_cpu / tcpu, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n_cpu} of {shots} syndromes, same inputs and windows, {tcpu:.1f} s",
               "paired_with_gpu_bit_exact": agree}
    wd.close()
    line = head(args, shots * args.steps / elapsed, elapsed, {
        "workload": "relay_bp_dem_936x8785_windowed", "matrix": "DEM-shaped synthetic 936x8785, 13 rounds of 72",
        "t_commit_rounds": tc, "t_overlap_rounds": to, "windows": nw, "shots": shots, "T_first": 80, "T_leg": 60,
        "legs": 20, "solutions": 1, "parallelism": "single_gpu"})
    line.update({"edge_updates_per_s": eu * args.steps / elapsed, "launch_ms": win_ms, "roofline": roof,
                 "lds_roofline": lds,
                 "ler": {"windowed": k_fail / shots, "wilson95": wilson(k_fail, shots),
                         "full_matrix": float(fail_full.mean()),
                         "all_windows_converged": float(conv.all(0).mean()),
                         "mean_iters_per_window": [float(x) for x in iters.mean(1)]},
                 "cpu_baseline": cpu})
    return line


# --------------------------------------------------------------------------
# plain-BP LLR export on the DEM-shaped matrix (25 rounds, gamma = 0)
# --------------------------------------------------------------------------


def run_bp_llr(args, torch, rb, codes, sampling):
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    prob = codes.dem_problem()
    M, N, E = prob.m, prob.n, prob.nnz
    shots = args.shots or 100000
    syn_np, _ = sampling.sample_syndromes_sparse(prob, 0xB9C5, shots)
    prm = rb.bp_params(25)
    dec = rb.Decoder.from_problem(prob, device=0, **prm)
    d_syn = torch.from_numpy(syn_np).to(dev)
    out = dec.decode(d_syn, want_llr=True)

    def step(ev):
        if ev is not None:
            ev[0][0].record(stream)
        dec.decode(d_syn, out=out)
        if ev is not None:
            ev[0][1].record(stream)

    elapsed, per_launch = timed(torch, step, 1, args.steps, args.warmup)
    kernel_ms = float(np.mean(per_launch))
    iters = out["iters"].cpu().numpy()
    conv = out["conv"].cpu().numpy()
    iters_launch = int(iters.astype(np.int64).sum())
    roof, lds = roofline("relay_block_kernel", kernel_ms, iters_launch * ops_per_iteration(M, N, E),
                         iters_launch * E, lds_bytes_per_edge_update(M, N, E), None)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle_threads()
        n_cpu = min(args.cpu_sample or 20000, shots)
        t1 = time.perf_counter()
        ref = oracle.decode(M, N, prob.rows, prob.cols, prob.prior, prm, syn_np[:n_cpu],
                            threads=threads, want_llr=True)
        tc = time.perf_counter() - t1
        agree = bool(np.array_equal(ref["llr"], out["llr"][:n_cpu].cpu().numpy())
                     and np.array_equal(ref["iters"], iters[:n_cpu]))
        cpu = {"value": n_cpu / tc, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n_cpu} of {shots} syndromes, same inputs, {tc:.1f} s",
               "paired_with_gpu_bit_exact": agree}
    line = head(args, shots * args.steps / elapsed, elapsed, {
        "workload": "plain_bp_llr_dem_936x8785", "matrix": "DEM-shaped synthetic 936x8785",
        "edges": E, "shots": shots, "rounds": 25, "gamma": 0.0, "legs": 1, "output": "llr f32 [B, N]",
        "parallelism": "single_gpu"})
    line.update({"edge_updates_per_s": iters_launch * E * args.steps / elapsed,
                 "launch_ms": [kernel_ms], "roofline": roof, "lds_roofline": lds,
                 "converged": float(conv.mean()), "mean_iters": float(iters.mean()),
                 "kernel_config": dec.info(), "cpu_baseline": cpu})
    return line


# --------------------------------------------------------------------------
# four BB codes interleaved 4:3:2:1: one mixed launch vs four per-code launches
# --------------------------------------------------------------------------


def run_mixed_codes(args, torch, rb, codes, sampling):
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    names = ("bb72", "bb90", "bb144", "bb288")
    pattern = np.array([0, 1, 2, 0, 3, 1, 0, 2, 1, 0], np.int32)  # 4:3:2:1
    shots = args.shots or 400000
    probs = [codes.bb_problem(nm, 0.04) for nm in names]
    code_id = np.resize(pattern, shots).astype(np.int32)
    m_max = max(p.m for p in probs)
    syn = np.zeros((shots, m_max), np.uint8)
    per = []
    for k, pr in enumerate(probs):
        idx = np.nonzero(code_id == k)[0]
        f, s = sampling.sample_batch(pr, (4 << 32) | k, 0, idx.size)
        syn[idx, :pr.m] = s
        per.append((idx, f, s))
    mdec = rb.MultiDecoder(probs, device=0, **RELAY_R20)
    d_code = torch.from_numpy(code_id).to(dev)
    d_syn = torch.from_numpy(syn).to(dev)
    mout = mdec.alloc(shots)
    samples = [torch.from_numpy(per[k][2][:20000]).to(dev) for k in range(len(probs))]
    chosen = mdec.autotune(samples, reps=2)

    def step_mixed(ev):
        if ev is not None:
            ev[0][0].record(stream)
        mdec.decode(d_code, d_syn, out=mout)
        if ev is not None:
            ev[0][1].record(stream)

    el_mixed, pl_mixed = timed(torch, step_mixed, 1, args.steps, args.warmup)
    host = {k: v.cpu().numpy() for k, v in mout.items() if k != "workspace"}
    # per-shot fixed cost: an all-zero syndrome converges at the first
    # iteration, so a batch of them costs one fetch, one check pass and one
    # convergence event per shot
    d_zero = torch.zeros_like(d_syn)
    zout = mdec.alloc(shots)

    def step_zero(ev):
        if ev is not None:
            ev[0][0].record(stream)
        mdec.decode(d_code, d_zero, out=zout)
        if ev is not None:
            ev[0][1].record(stream)

    _, pl_zero = timed(torch, step_zero, 1, max(2, args.steps // 2), 1)
    assert int(zout["iters"].max().item()) == 1
    del zout
    # the same launch captured in a hipGraph and replayed
    gout = mdec.alloc(shots)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        mdec.decode(d_code, d_syn, out=gout)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        mdec.decode(d_code, d_syn, out=gout)

    def step_graph(ev):
        if ev is not None:
            ev[0][0].record(stream)
        graph.replay()
        if ev is not None:
            ev[0][1].record(stream)

    el_graph, pl_graph = timed(torch, step_graph, 1, args.steps, args.warmup)
    graph_same = all(np.array_equal(gout[k].cpu().numpy(), host[k]) for k in host)
    del graph
    # four per-code launches, each code's syndromes contiguous, autotuned per code
    decs, d_per, outs = [], [], []
    for k, pr in enumerate(probs):
        d = rb.Decoder.from_problem(pr, device=0, **RELAY_R20)
        d.autotune(samples[k], reps=2)
        decs.append(d)
        d_per.append(torch.from_numpy(per[k][2]).to(dev))
        outs.append(d.decode(d_per[-1]))

    def step_per(ev):
        for k in range(len(probs)):
            if ev is not None:
                ev[k][0].record(stream)
            decs[k].decode(d_per[k], out=outs[k])
            if ev is not None:
                ev[k][1].record(stream)

    el_per, pl_per = timed(torch, step_per, len(probs), args.steps, args.warmup)
    ler, same = {}, True
    eu_launch, ops_launch = 0, 0.0
    for k, pr in enumerate(probs):
        idx, f, s = per[k]
        fail = logical_failures(pr, f, host["corr"][idx, :pr.n], host["conv"][idx])
        n_fail = int(fail.sum())
        it = int(host["iters"][idx].astype(np.int64).sum())
        ler[names[k]] = {"shots": int(idx.size), "ler": n_fail / idx.size,
                         "wilson95": wilson(n_fail, idx.size),
                         "mean_iters": float(host["iters"][idx].mean())}
        same &= bool(np.array_equal(outs[k]["corr"].cpu().numpy(), host["corr"][idx, :pr.n])
                     and np.array_equal(outs[k]["iters"].cpu().numpy(), host["iters"][idx]))
        eu_launch += it * pr.nnz
        ops_launch += it * ops_per_iteration(pr.m, pr.n, pr.nnz)
    kernel_ms = float(np.mean(pl_mixed))
    lds_b = sum(int(host["iters"][per[k][0]].astype(np.int64).sum()) * pr.nnz *
                lds_bytes_per_edge_update(pr.m, pr.n, pr.nnz)
                for k, pr in enumerate(probs)) / eu_launch
    roof, lds = roofline("relay_mixed_kernel", kernel_ms, ops_launch, eu_launch, lds_b,
                         stored_traffic("relay_mixed_kernel_mixed_bb_codes_hbm_traffic.txt"))
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle_threads()
        n_cpu = min(args.cpu_sample or 100000, shots)
        t1 = time.perf_counter()
        agree = True
        for k, pr in enumerate(probs):
            idx = per[k][0]
            sel = idx[idx < n_cpu]
            ref = oracle.decode(pr.m, pr.n, pr.rows, pr.cols, pr.prior, RELAY_R20, syn[sel, :pr.m],
                                threads=threads)
            agree &= bool(np.array_equal(ref["corr"], host["corr"][sel, :pr.n])
                          and np.array_equal(ref["iters"], host["iters"][sel]))
        tc = time.perf_counter() - t1
        cpu = {"value": n_cpu / tc, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n_cpu} of {shots} interleaved syndromes, same inputs, {tc:.1f} s",
               "paired_with_gpu_bit_exact": agree}
    line = head(args, shots * args.steps / el_mixed, el_mixed, {
        "workload": "relay_bp_mixed_bb_codes", "codes": list(names), "proportions": "4:3:2:1",
        "shots": shots, "p": 0.04, "legs": 20, "solutions": 1, "schedule": "mixed",
        "parallelism": "single_gpu"})
    line.update({
        "edge_updates_per_s": eu_launch * args.steps / el_mixed,
        "launch_ms": [kernel_ms], "roofline": roof, "lds_roofline": lds,
        "hipgraph_replay": {"value": shots * args.steps / el_graph,
                            "launch_ms": float(np.mean(pl_graph)),
                            "results_identical": graph_same},
        "per_code_launches": {"value": shots * args.steps / el_per,
                              "launch_ms": launch_means(pl_per),
                              "results_identical": same},
        "per_shot_fixed_cost": {"zero_syndrome_launch_ms": float(np.mean(pl_zero)),
                                "ns_per_shot": float(np.mean(pl_zero)) * 1e6 / shots,
                                "share_of_launch": float(np.mean(pl_zero)) / kernel_ms,
                                "mean_iters": float(host["iters"].mean())},
        "tiles_chosen": chosen, "ler": ler, "cpu_baseline": cpu})
    return line


# --------------------------------------------------------------------------
# learned first leg on [[144,12,12]] at p = 0.04
# --------------------------------------------------------------------------


def run_learned(args, torch, rb, codes, sampling):
    """Trains gamma_j and the prior scale through the unrolled first leg (batch
    4096 of fresh errors per step, checkpoints every 10 iterations, Adam), then
    decodes held-out shots with and without the learned first leg.  Four
    trainings: as configured (lr 1e-2, loss at T = 60); with a smaller step
    and the loss averaged over depths 5, 10, 20, 40, 60; lr 1e-2 with gamma_j
    bounded to the paper's range through a sigmoid; and the same with the
    scale held at 1 (at T = 60 its gradient is a sum that cancels to ~1e-8 of
    its terms, below FP32 resolution)."""
    from paper_2511_21660_amd import learn

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    prob = codes.bb_problem("bb144", 0.04)
    steps_train = args.train_steps or 2000
    batch = 4096
    tdec = rb.Decoder.from_problem(prob, device=0, **RELAY_R20)
    trainings = {"lr1e-2_T60": dict(lr=1e-2, t_iters=60),
                 "lr1e-3_T5-60": dict(lr=1e-3, t_iters=(5, 10, 20, 40, 60)),
                 "lr1e-2_T60_bounded": dict(lr=1e-2, t_iters=60, gamma_range=(-0.24, 0.66)),
                 "lr1e-2_T60_bounded_s1": dict(lr=1e-2, t_iters=60, gamma_range=(-0.24, 0.66),
                                               learn_scale=False)}
    learned, train_info = {}, {}
    for tag, kw in trainings.items():
        t0 = time.perf_counter()
        gamma, scale, hist = learn.train_first_leg(
            tdec, prob, lambda k: sampling.sample_batch(prob, (7 << 32) | k, 0, batch), steps=steps_train,
            ckpt_every=10, log_every=max(1, steps_train // 10),
            log=lambda m, tag=tag: print(f"# {tag} {m}", file=sys.stderr, flush=True), **kw)
        torch.cuda.synchronize()
        learned[tag] = (gamma, scale)
        train_info[tag] = {"seconds": time.perf_counter() - t0, "loss_first": hist[0][1],
                           "loss_last": hist[-1][1], "scale": scale, "gamma_mean": float(gamma.mean()),
                           "gamma_min": float(gamma.min()), "gamma_max": float(gamma.max())}
    shots = args.shots or 1000000
    f_ev, s_ev = sampling.sample_batch(prob, 0xE7A1, 0, shots)
    d_syn = torch.from_numpy(s_ev).to(dev)
    forms = {"relay": dict(RELAY_R20), "dmem_leg": dict(RELAY_R20, num_legs=1, iters_first=60)}
    res = {}
    for form, prm in forms.items():
        for tag in [None] + list(learned):
            dec = rb.Decoder.from_problem(prob, device=0, **prm)
            if tag is not None:
                dec.set_leg_gamma(1, learned[tag][0])
                dec.set_prior_scale(learned[tag][1])
            out = dec.decode(d_syn)

            def step(ev, dec=dec, out=out):
                if ev is not None:
                    ev[0][0].record(stream)
                dec.decode(d_syn, out=out)
                if ev is not None:
                    ev[0][1].record(stream)

            el, pl = timed(torch, step, 1, args.steps, args.warmup)
            conv = out["conv"].cpu().numpy()
            corr = out["corr"].cpu().numpy()
            fail = logical_failures(prob, f_ev, corr, conv)
            k = int(fail.sum())
            it = int(out["iters"].to(torch.int64).sum().item())
            kms = float(np.mean(pl))
            roof, lds = roofline("relay_group_kernel", kms, it * ops_per_iteration(prob.m, prob.n, prob.nnz),
                                 it * prob.nnz, lds_bytes_per_edge_update(prob.m, prob.n, prob.nnz), None)
            res[f"{form}/{tag or 'gamma0=0.125'}"] = {
                "syndromes_per_s": shots * args.steps / el, "launch_ms": kms,
                "ler": k / shots, "wilson95": wilson(k, shots), "conv": float(conv.mean()),
                "mean_iters": float(out["iters"].float().mean().item()), "roofline": roof}
            if form == "relay" and tag == "lr1e-2_T60_bounded_s1" and not args.no_cpu_baseline:
                import oracle

                g1, sc = learned[tag]

                def decode_sample(n, threads, g1=g1, sc=sc, corr=corr, out=out):
                    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, s_ev[:n],
                                        threads=threads, gamma1=g1, scale=sc)
                    return bool(np.array_equal(ref["corr"], corr[:n])
                                and np.array_equal(ref["iters"], out["iters"][:n].cpu().numpy()))

                res["cpu_baseline"] = oracle_baseline(decode_sample, shots, 20000, shots,
                                                      "held-out syndromes, learned first leg")
            dec.close()
    best = res["relay/lr1e-2_T60_bounded_s1"]
    line = head(args, best["syndromes_per_s"], shots * args.steps / best["syndromes_per_s"], {
        "workload": "relay_bp_bb144_learned_first_leg", "code": "[[144,12,12]] HX 72x144", "p": 0.04,
        "train_steps": steps_train, "batch": batch, "unrolled_iters": 60, "ckpt_every": 10,
        "optimizer": "adam", "eval_shots": shots, "legs": 20, "solutions": 1,
        "parallelism": "single_gpu"})
    cpu = res.pop("cpu_baseline", None)
    line.update({"decoders": res, "training": train_info, "roofline": best["roofline"], "cpu_baseline": cpu})
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default per workload)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["bb144", "dem", "dem-2gross", "dem-window", "mixed-codes", "learned",
                                           "bp-llr"],
                    default="dem")
    ap.add_argument("--train-steps", type=int, default=0, help="learned: Adam steps (default 2000)")
    ap.add_argument("--shots", type=int, default=0,
                    help="syndromes per p (bb144) or in total (default per workload)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle sample: syndromes per p (bb144) or in total (dem)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--f16-steps", type=int, default=3,
                    help="dem: timed launches of the binary16 decoder on the same syndromes; bb144: "
                         "decode them with binary16 messages for the LER comparison (0: skip)")
    ap.add_argument("--io-layout", choices=["bits32", "bytes"], default="bits32",
                    help="dem, dem-2gross: syndromes in and corrections out bit-packed in uint32 words "
                         "(default) or one byte per entry")
    ap.add_argument("--schedule", choices=["per-p", "per-p-lpt", "mixed"], default="mixed",
                    help="bb144 only.  per-p: one launch per p in input order; per-p-lpt: one "
                         "launch per p, shots longest-first; mixed: all four p in one launch "
                         "(one code context per p)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="after timing, run one plain device copy kernel of MB MiB (int32 "
                         "bitwise_not: reads and writes MB MiB) to scale HBM counters")
    args = ap.parse_args()
    if args.steps <= 0:
        args.steps = DEFAULT_STEPS[args.workload]

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(json.dumps({"error": "the decoder runs on one GPU (shots are independent; no multi-GPU path): run with --gpus 1"}))
        sys.exit(2)

    import torch

    from paper_2511_21660_amd import relaybp as rb
    from workloads import codes, sampling

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        sys.exit(1)
    run = {"bb144": run_bb144, "dem": run_dem, "dem-2gross": lambda *x: run_dem(*x, two_gross=True),
           "dem-window": run_dem_window,
           "mixed-codes": run_mixed_codes,
           "learned": run_learned, "bp-llr": run_bp_llr}[args.workload]
    line = run(args, torch, rb, codes, sampling)
    if line.get("cpu_baseline") and "host" not in line["cpu_baseline"]:
        line["cpu_baseline"]["host"] = host_cpu()
    if args.calibrate_copy > 0:
        n_el = args.calibrate_copy * (1 << 20) // 4
        src = torch.arange(n_el, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        line["copy_calibration_bytes_each_way"] = n_el * 4
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
