"""rb_decode_multi_noalloc (the mixed decode with the library's static
scratch in place of a caller workspace) against rb_decode_multi, through the
C ABI: two calls in a row on one context, the second with a smaller batch,
both bit-identical to the workspace entry point on the same inputs."""
import ctypes

import numpy as np
import pytest

from tests.conftest import RELAY_DEFAULT
from workloads import codes, sampling

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIX = ("bb72", "bb90", "bb144", "bb288")
PATTERN = np.array([0, 1, 2, 0, 3, 1, 0, 2, 1, 0], np.int32)


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2511_21660_amd import relaybp

    relaybp.load_library()
    return relaybp


def _inputs(probs, b, key):
    code_id = np.resize(PATTERN, b).astype(np.int32)
    syn = np.zeros((b, max(p.m for p in probs)), np.uint8)
    for k, pr in enumerate(probs):
        idx = np.nonzero(code_id == k)[0]
        syn[idx, :pr.m] = sampling.sample_batch(pr, key | k, 0, idx.size)[1]
    return torch.from_numpy(code_id).cuda(), torch.from_numpy(syn).cuda()


def _poison(out):
    for k, v in out.items():
        if k != "workspace":
            v.fill_(0x5A if v.dtype == torch.uint8 else 7)


def _host(out, code_id, ns):
    """Outputs on the host, with the entries past each row's own code length
    (undefined padding of [B, N_max] rows) zeroed."""
    res = {}
    n_of = np.asarray(ns)[code_id.cpu().numpy()]
    for k, v in out.items():
        if k == "workspace":
            continue
        h = v.cpu().numpy()
        if h.ndim == 2:
            h = np.where(np.arange(h.shape[1])[None, :] < n_of[:, None], h, 0)
        res[k] = h
    return res


def test_noalloc_matches_workspace_entry_point(rb):
    probs = [codes.bb_problem(n, 0.05) for n in MIX]
    dec = rb.MultiDecoder(probs, **dict(RELAY_DEFAULT, num_solutions=2))
    assert dec.noalloc_max_batch() > 10 ** 6
    for b, key in ((1500, 21 << 32), (350, 22 << 32)):      # second call smaller
        d_code, d_syn = _inputs(probs, b, key)
        ref = dec.decode(d_code, d_syn, want_llr=True)
        got = dec.alloc(b, want_llr=True)
        _poison(got)
        dec.decode_noalloc(d_code, d_syn, got)
        torch.cuda.synchronize()
        ns = [pr.n for pr in probs]
        r, g = _host(ref, d_code, ns), _host(got, d_code, ns)
        for k in r:
            np.testing.assert_array_equal(g[k], r[k], err_msg=f"B={b} {k}")
        assert r["conv"].mean() > 0.9
    dec.close()


def test_noalloc_rejects_oversized_batch_before_gpu_work(rb):
    probs = [codes.bb_problem(n, 0.05) for n in MIX[:2]]
    dec = rb.MultiDecoder(probs, **RELAY_DEFAULT)
    L = rb.load_library()
    bmax = dec.noalloc_max_batch()
    d_code, d_syn = _inputs(probs, 10, 23 << 32)
    out = dec.alloc(10)
    args = [dec._h, bmax + 1, rb._ptr(d_code), rb._ptr(d_syn), rb._ptr(out["corr"]), rb._ptr(out["conv"]),
            rb._ptr(out["legs"]), rb._ptr(out["iters"]), None, None, None]
    assert L.rb_decode_multi_noalloc(*args) == 7                     # RB_E_WORKSPACE
    assert b"exceeds the static scratch" in L.rb_last_error_message()
    args[1] = 0
    assert L.rb_decode_multi_noalloc(*args) == 0                     # empty batch: no-op
    single = rb.Decoder.from_problem(probs[0], **RELAY_DEFAULT)
    args[0], args[1] = single._h, 10
    assert L.rb_decode_multi_noalloc(*args) == 1                     # not a mixed context
    assert L.rb_noalloc_max_batch(single._h) == 0
    torch.cuda.synchronize()
    dec.close()
    single.close()
