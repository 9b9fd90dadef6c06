"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

Two drivers are built in a temporary directory and run:
  * sanitize_oracle_main.c: every entry point of the C oracle on generated
    problems (all precisions, anchors, S > 1, cutoffs, traces);
  * sanitize_plan_main.cpp: the library's host planner through rb_plan_check
    (CSR / CSC layouts, the gather tables of every kernel configuration, the
    bank-aware plans and their consistency checks) on bivariate-bicycle codes,
    irregular graphs with empty rows and columns, long rows and a banded
    detector-error-model-like matrix.  The library is compiled with the
    sanitizers on its host code only (-Xarch_host); device code is built as
    usual and never launched.
A sanitizer report ends the driver with a nonzero status."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2511_21660_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout[-3000:]}\n{res.stderr[-3000:]}"
    return res


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(HERE, "sanitize_oracle_main.c"), "-lm", "-o", exe])
    out = _run([exe]).stdout
    assert "failures: 0" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_planner_under_asan_ubsan(tmp_path):
    flags = ["-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-omit-frame-pointer", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]
    srcs = [os.path.join(CSRC, f) for f in ("relay_kernels.hip", "relay_block.hip", "relay_block16.hip",
                                            "relay_large.hip", "relay_train.hip", "relay_api.cpp")]
    srcs.append(os.path.join(HERE, "sanitize_plan_main.cpp"))
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]
    with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda so: _run([HIPCC, "-c", *flags, so[0], "-o", so[1]]), zip(srcs, objs)))
    exe = str(tmp_path / "plan_san")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", *objs, "-o", exe])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0")).stdout
    assert "failures: 0" in out
