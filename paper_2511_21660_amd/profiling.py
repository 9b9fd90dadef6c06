"""Summaries of rocprofv3 output for the decoding kernels.

* ``stats``   : markdown table of a ``--kernel-trace --stats`` kernel_stats.csv.
* ``traffic`` : HBM bytes per launch of a kernel from two ``--pmc`` runs
  (FETCH_SIZE, WRITE_SIZE, both in KiB per dispatch), each scaled by what the
  same counter reads for a plain copy kernel that moves a known number of
  bytes each way; stamped with a hash of the kernel sources so that a stale
  figure is recognised after the kernels change.

* ``counters``: VALU and LDS activity of a kernel from one ``--pmc`` run of
  SQ counters (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_INSTS_LDS,
  SQ_LDS_BANK_CONFLICT, SQ_LDS_IDX_ACTIVE, SQ_WAIT_INST_LDS, SQ_BUSY_CU_CYCLES,
  GRBM_GUI_ACTIVE), normalised by the edge-updates of one launch:
    - cycles of a launch: GRBM_GUI_ACTIVE / XCDs (the counter sums the XCDs);
    - VALU busy: 4 SQ_ACTIVE_INST_VALU / (SIMDs x cycles) (quad-cycles, one
      per wave64 VALU instruction on a 16-lane SIMD);
    - lane-ops per edge-update: 64 SQ_INSTS_VALU / edge-updates (against the
      algorithmic count of the update rules);
    - LDS instructions per edge-update: 64 SQ_INSTS_LDS / edge-updates;
    - LDS active: SQ_LDS_IDX_ACTIVE / (CUs x cycles); bank-conflict share:
      SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE.

Usage (after the rocprofv3 runs):
    python -m paper_2511_21660_amd.profiling stats KERNEL_STATS_CSV
    python -m paper_2511_21660_amd.profiling traffic --fetch FETCH_CSV --write WRITE_CSV \
        --kernel relay_mixed_kernel --copy-kernel elementwise --copy-bytes N --out OUT_JSON
    python -m paper_2511_21660_amd.profiling counters --sq SQ_CSV --kernel relay_block_kernel \
        --edge-updates EU --ops-per-edge-update OPS [--launches-skip 0]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))


def _code_only(text: str) -> str:
    """Source text without comments and blank lines, so that editing a
    comment leaves the hash of a measured build unchanged (a rough cut: a
    "//" inside a string literal also starts a comment here, which only
    makes two such sources hash alike)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (ln.split("//", 1)[0].rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def source_hash() -> str:
    """SHA-256 over the code of the library's kernel and host sources
    (comments and blank lines left out)."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(_HERE, "csrc", "*"))):
        with open(path, encoding="utf-8") as f:
            h.update(os.path.basename(path).encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def stats_table(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def _counter_means(path: str, counter: str):
    sums = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        sums.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in sums.items()}


def _pick(means: dict, substr: str) -> float:
    hits = [v for k, v in means.items() if substr in k]
    if not hits:
        raise SystemExit(f"no kernel matching {substr!r} in counter output")
    return max(hits)


def traffic(fetch_csv, write_csv, kernel, copy_kernel, copy_bytes):
    f = _counter_means(fetch_csv, "FETCH_SIZE")
    w = _counter_means(write_csv, "WRITE_SIZE")
    fetch_scale = copy_bytes / (_pick(f, copy_kernel) * 1024.0)
    write_scale = copy_bytes / (_pick(w, copy_kernel) * 1024.0)
    fb = _pick(f, kernel) * 1024.0 * fetch_scale
    wb = _pick(w, kernel) * 1024.0 * write_scale
    return {"kernel": kernel, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
            "traffic_bytes_per_launch": fb + wb, "fetch_scale": fetch_scale,
            "write_scale": write_scale, "source_hash": source_hash()}


def _counter_rows(path: str, kernel: str):
    """{counter: [value per dispatch]} of the dispatches whose kernel name
    contains `kernel` (rows of one dispatch share its Dispatch_Id)."""
    per = {}
    for r in csv.DictReader(open(path)):
        if kernel not in r["Kernel_Name"]:
            continue
        per.setdefault(r["Dispatch_Id"], {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return [per[k] for k in sorted(per, key=int)]


def counters(sq_csv, kernel, edge_updates, ops_per_eu, cus=256, simds_per_cu=4, xcds=8, skip=0, near_max=0.9):
    """Derived VALU / LDS activity per launch, averaged over the dispatches
    (after `skip`) whose SQ_INSTS_VALU is at least `near_max` of the largest
    (the workload's own launches, not autotuning trials or smaller probes),
    for a launch of `edge_updates` edge-updates."""
    rows = _counter_rows(sq_csv, kernel)[skip:]
    if not rows:
        raise SystemExit(f"no dispatch of {kernel!r} in {sq_csv}")
    top = max(r["SQ_INSTS_VALU"] for r in rows)
    rows = [r for r in rows if r["SQ_INSTS_VALU"] >= near_max * top]
    mean = {k: sum(r[k] for r in rows) / len(rows) for k in rows[0]}
    cyc = mean["GRBM_GUI_ACTIVE"] / xcds
    out = {"kernel": kernel, "dispatches": len(rows), "cycles_per_launch": cyc,
           "valu_busy": 4.0 * mean["SQ_ACTIVE_INST_VALU"] / (cus * simds_per_cu * cyc),
           "lane_ops_per_edge_update": 64.0 * mean["SQ_INSTS_VALU"] / edge_updates,
           "algorithmic_ops_per_edge_update": ops_per_eu,
           "lds_instructions_per_edge_update": 64.0 * mean["SQ_INSTS_LDS"] / edge_updates,
           "lds_active": mean["SQ_LDS_IDX_ACTIVE"] / (cus * cyc),
           "lds_bank_conflict_share": mean["SQ_LDS_BANK_CONFLICT"] / max(1.0, mean["SQ_LDS_IDX_ACTIVE"]),
           "raw_means": mean, "source_hash": source_hash()}
    out["algorithmic_share_of_valu"] = ops_per_eu / out["lane_ops_per_edge_update"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-kernel", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--sq", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--edge-updates", type=float, required=True)
    c.add_argument("--ops-per-edge-update", type=float, required=True)
    c.add_argument("--launches-skip", type=int, default=0)
    c.add_argument("--near-max", type=float, default=0.9)
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        print(json.dumps(counters(a.sq, a.kernel, a.edge_updates, a.ops_per_edge_update, skip=a.launches_skip,
                                  near_max=a.near_max), indent=1))
        return 0
    if a.cmd == "stats":
        print(stats_table(a.csv))
    else:
        res = traffic(a.fetch, a.write, a.kernel, a.copy_kernel, a.copy_bytes)
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
