"""LDS read bandwidth of the GPU, measured (the peak of the LDS roofline).

Runs the probe of ``csrc/lds_peak.hip`` (conflict-free ds_read_b32, _b64 and
_b128 loops, 256-thread workgroups with 16 KiB of LDS each, eight per CU)
and reports, per width, the bytes read per second, the shader clock the
reads ran at (from the probe's clock64 / wall_clock64 pair) and the bytes
per CU per clock.

    python -m paper_2511_21660_amd.ldspeak [--blocks-per-cu 8] [--iters 65536]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, "liblds_peak.so")


def measure(blocks_per_cu=8, iters=65536, reps=5):
    import torch

    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    lib.lds_peak_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P,
                                 ctypes.POINTER(ctypes.c_float)]
    lib.lds_peak_run.restype = ctypes.c_int
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    blocks = cus * blocks_per_cu
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    clk = torch.empty(blocks * 2, dtype=torch.int64, device="cuda")
    res = {"cus": cus, "blocks": blocks, "threads_per_block": 256, "iters": iters, "widths": {}}
    lib.lds_peak_wall_clock_khz.argtypes = [ctypes.c_int]
    lib.lds_peak_wall_clock_khz.restype = ctypes.c_int
    wall_hz = lib.lds_peak_wall_clock_khz(0) * 1e3
    if wall_hz <= 0:
        raise RuntimeError("wall clock rate unavailable")
    for width in (4, 8, 16):
        ms = ctypes.c_float(0.0)
        rc = lib.lds_peak_run(width, blocks, iters, reps, P(out.data_ptr()), P(clk.data_ptr()),
                              ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"lds_peak_run({width}) failed with {rc}")
        torch.cuda.synchronize()
        c = clk.view(blocks, 2).cpu().double()
        ghz = float((c[:, 0] / c[:, 1]).median()) * wall_hz / 1e9
        bytes_ = float(blocks) * 256 * iters * width
        tbs = bytes_ / (ms.value * 1e-3) / 1e12
        res["widths"][f"ds_read_b{8 * width}"] = {
            "ms": ms.value, "bytes": bytes_, "TB_per_s": tbs, "shader_clock_GHz": ghz,
            "bytes_per_clk_per_cu": tbs * 1e12 / (cus * ghz * 1e9),
            "TB_per_s_at_2p4GHz": tbs * 1e12 / (cus * ghz * 1e9) * cus * 2.4e9 / 1e12}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks-per-cu", type=int, default=8)
    ap.add_argument("--iters", type=int, default=65536)
    a = ap.parse_args()
    print(json.dumps(measure(a.blocks_per_cu, a.iters)))


if __name__ == "__main__":
    main()
