"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the public header declares, and rejects invalid arguments on
the host before touching the device."""
import ctypes

import numpy as np
import pytest

from paper_2511_21660_amd import relaybp as rb
from workloads import codes


@pytest.fixture(scope="module")
def lib():
    return rb.load_library()


def test_exports_every_header_symbol(lib):
    names = rb.header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/relaybp.h but not exported"


def test_status_strings(lib):
    for code in range(11):
        s = lib.rb_status_string(code)
        assert s and s != b"unknown status"
    assert lib.rb_status_string(99) == b"unknown status"


def test_params_default_matches_paper(lib):
    p = rb.default_params()
    # appendix on Relay resources: T = 80 then 60, gamma_0 = 0.125,
    # gamma ~ U[-0.24, 0.66], 300 legs after the first (301 in total)
    assert (p.num_legs, p.iters_first, p.iters_leg, p.num_solutions) == (301, 80, 60, 1)
    assert p.gamma_first == np.float32(0.125)
    assert (p.gamma_lo, p.gamma_hi) == (np.float32(-0.24), np.float32(0.66))
    assert p.llr_clip == 2.0 ** 64
    assert p.io_layout == rb.IO_BYTES
    assert lib.rb_params_default(None) == 1


def _create(m, n, rows, cols, prior, params=None):
    lib = rb.load_library()
    h = ctypes.c_void_p()
    rows = np.ascontiguousarray(rows, np.int32)
    cols = np.ascontiguousarray(cols, np.int32)
    prior = np.ascontiguousarray(prior, np.float64)
    params = params or rb.default_params()
    st = lib.rb_create(ctypes.byref(h), m, n, rows.size, rows.ctypes.data_as(ctypes.c_void_p),
                       cols.ctypes.data_as(ctypes.c_void_p), prior.ctypes.data_as(ctypes.c_void_p),
                       ctypes.byref(params), 0)
    if st == 0:
        lib.rb_destroy(h)
    return st, lib.rb_last_error_message().decode()


def test_create_rejects_bad_input_before_device_use():
    p = codes.bb_problem("bb72", 0.05)
    assert _create(0, p.n, p.rows, p.cols, p.prior)[0] == 2
    assert _create(p.m, 0, p.rows, p.cols, np.zeros(0))[0] == 2
    rows = p.rows.copy()
    rows[3] = p.m
    assert _create(p.m, p.n, rows, p.cols, p.prior)[0] == 2
    cols = p.cols.copy()
    cols[0] = -1
    assert _create(p.m, p.n, p.rows, cols, p.prior)[0] == 2
    dup_r = np.concatenate([p.rows, p.rows[:1]])
    dup_c = np.concatenate([p.cols, p.cols[:1]])
    st, msg = _create(p.m, p.n, dup_r, dup_c, p.prior)
    assert st == 3 and "duplicate" in msg
    for bad in (0.0, 1.0, -0.1, np.nan, np.inf):
        prior = p.prior.copy()
        prior[5] = bad
        assert _create(p.m, p.n, p.rows, p.cols, prior)[0] == 4
    for field, val in (("num_legs", 0), ("iters_first", 0), ("iters_leg", -1),
                       ("num_solutions", 0), ("anchor", 2), ("max_total_iters", -1),
                       ("llr_clip", 0.0), ("gamma_lo", 1.0), ("io_layout", 2), ("io_layout", -1),
                       ("precision", 2), ("precision", -1)):
        assert _create(p.m, p.n, p.rows, p.cols, p.prior, rb.default_params(**{field: val}))[0] == 1
    assert _create(p.m, p.n, p.rows, p.cols, p.prior,
                   rb.default_params(gamma_first=float("nan")))[0] == 9


def test_mixed_launch_rejects_binary16_before_device_use():
    p = codes.bb_problem("bb72", 0.05)
    rows = np.ascontiguousarray(p.rows, np.int32)
    cols = np.ascontiguousarray(p.cols, np.int32)
    prior = np.ascontiguousarray(p.prior, np.float64)
    desc = (rb.RBCodeDesc * 1)(rb.RBCodeDesc(p.m, p.n, rows.size, rows.ctypes.data_as(ctypes.c_void_p),
                                             cols.ctypes.data_as(ctypes.c_void_p),
                                             prior.ctypes.data_as(ctypes.c_void_p)))
    h = ctypes.c_void_p()
    lib = rb.load_library()
    st = lib.rb_create_multi(ctypes.byref(h), 1, desc, ctypes.byref(rb.default_params(precision=rb.PREC_F16)), 0)
    assert st == 8 and b"FP32" in lib.rb_last_error_message()


def test_create_on_gpu_less_host_reports_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = codes.bb_problem("bb72", 0.05)
    st, msg = _create(p.m, p.n, p.rows, p.cols, p.prior)
    assert st == 5 and msg


def test_unsupported_graph_is_reported():
    import torch

    if torch.cuda.is_available():
        pytest.skip("checked on CPU hosts only")
    # 40,000 faults exceed every built-in configuration (the large-graph
    # kernel keeps Lambda of at most 32,768 faults in LDS)
    n = 40000
    st, msg = _create(1, n, np.zeros(n, np.int32), np.arange(n, dtype=np.int32), np.full(n, 0.1))
    assert st == 8 and "exceeds" in msg


def test_null_arguments(lib):
    assert lib.rb_create(None, 1, 1, 0, None, None, None, None, 0) == 1
    assert lib.rb_decode(None, 1, None, None, None, None, None, None, None, None) == 1
    assert lib.rb_trace(None, 1, None, None, ctypes.c_float(1.0), 1, None, None) == 1
    assert lib.rb_get_info(None, None) == 1
    assert lib.rb_sync_status(None) == 1
    assert lib.rb_syndrome(None, 1, None, None, None, None) == 1
    assert lib.rb_decode_multi_noalloc(None, 1, None, None, None, None, None, None, None, None, None) == 1
    assert lib.rb_noalloc_max_batch(None) == 0
    assert lib.rb_set_code_variant(None, 0, 0) == 1
    lib.rb_destroy(None)


_OOM_CHILD = r"""
import ctypes, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2511_21660_amd import relaybp as rb
L = rb.load_library()
# a valid 20000 x 20000 graph of 2x10^7 distinct entries (1000 per row)
k = np.arange(20_000_000, dtype=np.int64)
rows = (k // 1000).astype(np.int32)
cols = ((k % 1000) * 20 + (k // 1000) % 20).astype(np.int32)
rep = rb.RBPlanReport()
# cap the address space a little above what the process holds now, so the
# library's 160 MB of sorted entry pairs cannot be allocated
vm = int([l.split()[1] for l in open("/proc/self/status") if l.startswith("VmSize:")][0]) * 1024
resource.setrlimit(resource.RLIMIT_AS, (vm + (32 << 20), resource.RLIM_INFINITY))
st = L.rb_plan_check(20000, 20000, rows.size, rows.ctypes.data_as(ctypes.c_void_p),
                     cols.ctypes.data_as(ctypes.c_void_p), -1, ctypes.byref(rep))
print(st, L.rb_last_error_message().decode(), flush=True)
"""


def test_host_allocation_failure_returns_oom_instead_of_aborting(tmp_path):
    """A host allocation that fails inside the library (here: the sorted entry
    list of a large graph, under an address-space cap) comes back as
    RB_E_OOM with a message; no C++ exception crosses the C ABI."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "oom_child.py"
    script.write_text(_OOM_CHILD)
    res = subprocess.run([sys.executable, str(script), root], capture_output=True, text=True, timeout=120,
                         env=dict(os.environ, OMP_NUM_THREADS="1"))
    assert res.returncode == 0, res.stderr[-2000:]
    status, msg = res.stdout.strip().split(" ", 1)
    assert int(status) == 6 and "allocation" in msg, res.stdout
