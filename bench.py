#!/usr/bin/env python3
"""Relay-BP decoding throughput on one MI355X.

Default workload: plain Relay-BP FP32 on the [[144,12,12]] bivariate-bicycle
code (HX 72 x 144, E = 432 edges), i.i.d. code-capacity faults at
p in {0.02, 0.04, 0.06, 0.08}, 10^5 syndromes per p, T_1 = 80, T_r = 60,
R = 301 legs in total, S = 5 solutions kept (lowest weight output).
One step = decoding all 4 x 10^5 syndromes (four launches, one decoder per p),
syndromes already resident in HBM.

Prints one JSON line: syndromes/s (the headline), edge-updates/s, the roofline
of the decode kernel measured with HIP events on the launch stream, and the
CPU oracle timed on a bounded sample of the same workload on the host cores.
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
PEAK_LDS_TBS = 256 * 128 * 2.4e9 / 1e12       # 78.6 TB/s at 128 B/clk/CU
PEAK_HBM_GBS = 8000.0

RELAY = dict(num_legs=301, iters_first=80, iters_leg=60, num_solutions=5, gamma_first=0.125,
             gamma_lo=-0.24, gamma_hi=0.66, llr_clip=2.0 ** 64, seed=0x52454C4159, anchor=0,
             max_total_iters=0)

# Algorithmic work per edge-update (one edge in one iteration), from the
# update rules: check side nu = clip(Lambda - mu) (2), sign parity (1),
# min1/min2 tracking (3), per-edge magnitude select (2) and sign (1); fault
# side sum (1); syndrome parity (1) => 11 per edge, plus per fault 7
# (1 - gamma, two products, sum, two clips, decision) and per check 3.
OPS_PER_EDGE = 11.0
OPS_PER_FAULT = 7.0
OPS_PER_CHECK = 3.0


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shots", type=int, default=100000, help="syndromes per p")
    ap.add_argument("--cpu-sample", type=int, default=100000, help="oracle shots per p")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--schedule", choices=["per-p", "per-p-lpt", "mixed"], default="mixed",
                    help="per-p: one launch per p in input order; per-p-lpt: one launch per p, "
                         "shots longest-first; mixed: all four p in one launch (one code "
                         "context per p), longest-first per p")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="after timing, run one plain device copy kernel of MB MiB (int32 "
                         "bitwise_not: reads and writes MB MiB) to scale HBM counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(json.dumps({"error": "this build decodes on one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch

    from paper_2511_21660_amd import relaybp as rb
    from workloads import codes, sampling

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        sys.exit(1)
    dev = torch.device("cuda", 0)
    ps = [0.02, 0.04, 0.06, 0.08]
    probs, faults, syns = [], [], []
    for q, p in enumerate(ps):
        prob = codes.bb_problem("bb144", p)
        f, s = sampling.sample_batch(prob, (2 << 32) | q, 0, args.shots)
        probs.append(prob)
        faults.append(f)
        syns.append(s)
    E = probs[0].nnz
    stream = torch.cuda.current_stream(dev)
    if args.schedule == "mixed":
        mdec = rb.MultiDecoder(probs, device=0, **RELAY)
        code_id = torch.cat([torch.full((s.shape[0],), q, dtype=torch.int32)
                             for q, s in enumerate(syns)]).to(dev)
        d_all = torch.from_numpy(np.concatenate(syns)).to(dev)
        mout = mdec.alloc(d_all.shape[0])
        decs = None
        offs = np.cumsum([0] + [s.shape[0] for s in syns])

        def step(events=None):
            if events is not None:
                events[0][0].record(stream)
            mdec.decode(code_id, d_all, out=mout)
            if events is not None:
                events[0][1].record(stream)

        n_launch = 1

        def results():
            host = {k: v.cpu().numpy() for k, v in mout.items() if k != "workspace"}
            return [{k: v[offs[q]:offs[q + 1]] for k, v in host.items()} for q in range(len(ps))]
    else:
        decs = [rb.Decoder.from_problem(pr, device=0, **RELAY) for pr in probs]
        for d in decs:
            if args.variant is not None:
                d.set_variant(args.variant)
            if args.schedule == "per-p-lpt":
                d.reserve(args.shots)
        d_syn = [torch.from_numpy(s).to(dev) for s in syns]
        outs = []
        for s in syns:
            b = s.shape[0]
            outs.append({
                "corr": torch.empty((b, 144), dtype=torch.uint8, device=dev),
                "conv": torch.empty(b, dtype=torch.uint8, device=dev),
                "legs": torch.empty(b, dtype=torch.int32, device=dev),
                "iters": torch.empty(b, dtype=torch.int32, device=dev),
                "weight": torch.empty(b, dtype=torch.float64, device=dev),
            })

        def step(events=None):
            for q in range(len(ps)):
                if events is not None:
                    events[q][0].record(stream)
                decs[q].decode(d_syn[q], out=outs[q])
                if events is not None:
                    events[q][1].record(stream)

        n_launch = len(ps)

        def results():
            return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    launch_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n_launch)]
        step(ev)
        launch_ms.append(ev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_launch = [[e[0].elapsed_time(e[1]) for e in evs] for evs in launch_ms]
    kernel_ms = float(np.mean(per_launch))

    res = results()
    n_shots = sum(s.shape[0] for s in syns)
    iters_total = sum(int(r["iters"].astype(np.int64).sum()) for r in res)
    edge_updates_step = iters_total * E
    value = n_shots * args.steps / elapsed
    eu_per_s = edge_updates_step * args.steps / elapsed

    # roofline of the decode kernel: algorithmic ops per launch / mean launch time
    per_launch_eu = [int(r["iters"].astype(np.int64).sum()) * E for r in res]
    if n_launch == 1:
        per_launch_eu = [sum(per_launch_eu)]
    ops_per_iter = OPS_PER_EDGE * E + OPS_PER_FAULT * 144 + OPS_PER_CHECK * 72
    ops_launch = np.mean([eu / E * ops_per_iter for eu in per_launch_eu])
    achieved_tops = ops_launch / (kernel_ms * 1e-3) / 1e12
    b_alg = 8.0 + (8.0 * 144 + 12.0 * 72) / E
    lds_tbs = np.mean(per_launch_eu) * b_alg / (kernel_ms * 1e-3) / 1e12

    ler = {}
    for q, p in enumerate(ps):
        fail = logical_failures(probs[q], faults[q], res[q]["corr"], res[q]["conv"])
        k = int(fail.sum())
        ler[str(p)] = {"ler": k / len(fail), "wilson95": wilson(k, len(fail)),
                       "conv": float(res[q]["conv"].mean()),
                       "mean_iters": float(res[q]["iters"].mean()),
                       "max_iters": int(res[q]["iters"].max())}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = min(16, os.cpu_count() or 1)
        n_cpu = min(args.cpu_sample, args.shots)
        t1 = time.perf_counter()
        agree = True
        for q in range(len(ps)):
            ref = oracle.decode(probs[q].m, probs[q].n, probs[q].rows, probs[q].cols,
                                probs[q].prior, RELAY, syns[q][:n_cpu], threads=threads)
            agree &= bool(np.array_equal(ref["corr"], res[q]["corr"][:n_cpu])
                          and np.array_equal(ref["iters"], res[q]["iters"][:n_cpu]))
        tc = time.perf_counter() - t1
        cpu = {"value": 4 * n_cpu / tc, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n_cpu} syndromes of each of the 4 p values "
                         f"({4 * n_cpu} of {n_shots}), same inputs, {tc:.1f} s",
               "paired_with_gpu_bit_exact": agree}

    copy_bytes = 0
    if args.calibrate_copy > 0:
        n_el = args.calibrate_copy * (1 << 20) // 4
        src = torch.arange(n_el, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        copy_bytes = n_el * 4

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "relay_mixed_kernel_bb144_hbm_traffic.txt")
    if args.schedule == "mixed" and os.path.exists(tpath):
        from paper_2511_21660_amd import profiling

        rec = json.load(open(tpath))
        if rec.get("source_hash") == profiling.source_hash():
            traffic = rec["traffic_bytes_per_launch"]

    info = decs[0].info() if decs else {"variant": "mixed", "lanes_per_shot": None,
                                         "checks_per_lane": None, "cols_per_lane": None,
                                         "shots_per_block": None, "lds_bytes_per_block": None,
                                         "blocks_per_cu": None, "grid_blocks": None}
    line = {
        "metric": "syndromes decoded/s at matched LER; edge-updates/s and % HBM/LDS roofline",
        "value": value,
        "unit": "syndromes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "relay_bp_bb144_code_capacity",
                   "code": "[[144,12,12]] HX 72x144", "edges": E,
                   "p": ps, "syndromes_per_p": args.shots, "syndromes_per_step": n_shots,
                   "T_first": 80, "T_leg": 60, "legs": 301, "solutions": 5,
                   "gamma_first": 0.125, "gamma_range": [-0.24, 0.66], "anchor": "chain",
                   "schedule": args.schedule, "parallelism": "single_gpu"},
        "edge_updates_per_s": eu_per_s,
        "launch_ms": [float(np.mean([pl[q] for pl in per_launch])) for q in range(n_launch)],
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": PEAK_VALU_TOPS,
                     "unit": "Tops/s", "frac": achieved_tops / PEAK_VALU_TOPS, "traffic": traffic,
                     "kernel": ("relay_mixed_kernel" if args.schedule == "mixed"
                                else "relay_group_kernel"),
                     "kernel_ms_per_launch": kernel_ms,
                     "ops_per_edge_update": ops_per_iter / E},
        "lds_roofline": {"achieved": lds_tbs, "peak": PEAK_LDS_TBS, "unit": "TB/s",
                         "frac": lds_tbs / PEAK_LDS_TBS, "bytes_per_edge_update": b_alg},
        "ler": ler,
        "kernel_config": {k: info[k] for k in ("variant", "lanes_per_shot", "checks_per_lane",
                                               "cols_per_lane", "shots_per_block",
                                               "lds_bytes_per_block", "blocks_per_cu",
                                               "grid_blocks")},
        "cpu_baseline": cpu,
    }
    if copy_bytes:
        line["copy_calibration_bytes_each_way"] = copy_bytes
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
