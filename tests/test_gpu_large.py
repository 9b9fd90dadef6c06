"""GPU parity of the large-graph kernel (compressed check messages in LDS)
against the CPU oracle: bit-exact corrections, converged flags, leg and
iteration counts, weights and FP32 marginals.

The kernel serves graphs whose per-edge messages do not fit in LDS, up to a
two-gross-scale 2736 x 26208 matrix; it is also run here on the 936 x 8785
DEM-shaped matrix (where the block kernel is the default) and on irregular
graphs with empty rows and columns, by selecting its configuration."""
import numpy as np
import pytest

import oracle
from tests.conftest import RELAY_DEFAULT
from tests.test_gpu_parity import KEYS, _irregular_problem, assert_parity, gpu_decode
from workloads import codes, sampling

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2511_21660_amd import relaybp

    relaybp.load_library()
    return relaybp


@pytest.fixture(scope="module")
def dem():
    return codes.dem_problem()


def _large_variants(rb, prob):
    """Configuration indices of the large-graph kernel that fit `prob`."""
    nvar = rb.Decoder.from_problem(prob, **RELAY_DEFAULT)
    n = nvar.info()["num_variants"]
    nvar.close()
    out = []
    for v in range(n):
        r = None
        try:
            r = rb.plan_check(prob.m, prob.n, prob.rows, prob.cols, v)
        except rb.RelayError as e:
            assert e.status == 8
        if r is not None and r["block_kernel"] == 2:
            out.append(v)
    return out


def test_dem_on_large_kernel(rb, dem):
    """936 x 8785 DEM (rows up to degree 63) on both large-graph shapes: 160
    shots, R = 20, S = 1, bit-exact against the oracle."""
    _, syn = sampling.sample_batch(dem, 3 << 32, 0, 160)
    ref = oracle.decode(dem.m, dem.n, dem.rows, dem.cols, dem.prior, RELAY_DEFAULT, syn, want_llr=True)
    vs = _large_variants(rb, dem)
    assert len(vs) == 2
    for v in vs:
        gpu = gpu_decode(rb, dem, RELAY_DEFAULT, syn, variant=v)
        assert gpu["info"]["threads_per_block"] == 1024
        assert_parity(gpu, ref, syn, dem, f"dem large variant {v}")


def test_dem_large_kernel_prior_anchor_solutions_cutoff(rb, dem):
    _, syn = sampling.sample_batch(dem, 5 << 32, 0, 100)
    prm = dict(RELAY_DEFAULT, anchor=1, num_solutions=3, num_legs=8, max_total_iters=300)
    ref = oracle.decode(dem.m, dem.n, dem.rows, dem.cols, dem.prior, prm, syn, want_llr=True)
    gpu = gpu_decode(rb, dem, prm, syn, variant=_large_variants(rb, dem)[0])
    assert_parity(gpu, ref, syn, dem, "dem large prior anchor S=3 cutoff")


def test_dem_large_kernel_trace(rb, dem):
    """Message-level hook: 25 iterations of one leg with per-column gamma and
    a scaled prior, every marginal equal to the oracle's."""
    _, syn = sampling.sample_batch(dem, 17, 0, 4)
    gamma = np.random.default_rng(9).uniform(-0.24, 0.66, dem.n).astype(np.float32)
    dec = rb.Decoder.from_problem(dem, **RELAY_DEFAULT)
    dec.set_variant(_large_variants(rb, dem)[0])
    tr = dec.trace(torch.from_numpy(syn).cuda(), torch.from_numpy(gamma).cuda(), 25, scale=0.8).cpu().numpy()
    dec.close()
    ref = oracle.trace(dem.m, dem.n, dem.rows, dem.cols, dem.prior, gamma, 25, syn, scale=0.8)
    np.testing.assert_array_equal(tr, ref)


@pytest.mark.parametrize("seed", [1, 3])
def test_irregular_graphs_on_large_kernel(rb, seed):
    """Empty rows and columns, a degree-1 check, erasure priors, all-zero and
    all-one syndromes, S = 2, on the large-graph kernel."""
    prob = _irregular_problem(seed)
    _, syn = sampling.sample_batch(prob, 40 + seed, 0, 200)
    syn[:3] = 0
    syn[3:6] = 1
    prm = dict(RELAY_DEFAULT, num_solutions=2, num_legs=10)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn, want_llr=True)
    for v in _large_variants(rb, prob):
        gpu = gpu_decode(rb, prob, prm, syn, variant=v)
        assert_parity(gpu, ref, syn, prob, f"irregular seed={seed} large variant {v}")


def test_long_rows_over_several_check_records(rb):
    """Rows of degree 1..90 side by side: long rows span up to three 16-byte
    check records (state and 32 sign bits each), short rows sit between them
    in records written by other threads; uniform priors make many |nu| tie
    at the first iteration."""
    rng = np.random.default_rng(21)
    m, n = 300, 2400
    rows, cols = [], []
    for i in range(m):
        d = int(rng.integers(1, 91)) if i % 3 else int(rng.integers(1, 4))
        for j in rng.choice(n, d, replace=False):
            rows.append(i)
            cols.append(j)
    h = np.zeros((m, n), np.uint8)
    h[np.array(rows), np.array(cols)] = 1
    prob = codes.problem_from_dense("long_rows", h, np.full(n, 0.03), np.zeros((1, n), np.uint8))
    _, syn = sampling.sample_batch(prob, 8, 0, 96)
    prm = dict(RELAY_DEFAULT, num_legs=6)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn, want_llr=True)
    vs = _large_variants(rb, prob)
    assert vs
    gpu = gpu_decode(rb, prob, prm, syn, variant=vs[0])
    assert_parity(gpu, ref, syn, prob, "long rows on the large kernel")


def test_two_gross_scale_dem(rb):
    """2736 x 26208 DEM-shaped matrix (82.6K edges, rows up to degree 81): the
    large-graph kernel is the configuration chosen; 400 shots decoded, every
    converged correction valid, 128 sampled shots bit-exact against the
    oracle (R = 20, S = 1)."""
    prob = codes.dem_problem(2736, 26208)
    _, syn = sampling.sample_batch(prob, 6 << 32, 0, 400)
    gpu = gpu_decode(rb, prob, RELAY_DEFAULT, syn)
    assert gpu["info"]["threads_per_block"] == 1024 and gpu["info"]["checks_per_lane"] == 3
    h = prob.dense().astype(np.int64)
    ok = (gpu["corr"].astype(np.int64) @ h.T) % 2 == (syn != 0)
    assert ok[gpu["conv"] == 1].all() and gpu["conv"].mean() > 0.3
    idx = np.random.default_rng(2).choice(len(syn), 128, replace=False)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, RELAY_DEFAULT, syn[idx],
                        want_llr=True)
    sub = {k: gpu[k][idx] for k in KEYS}
    sub["info"] = gpu["info"]
    assert_parity(sub, ref, syn[idx], prob, "two-gross sample")


def test_two_gross_full_size_validity_and_sampled_parity(rb):
    """The two-gross-scale workload at full size, in the launch configuration
    the benchmark times (the same 2x10^5 seeded syndromes, bit-packed in and
    out, R = 20, S = 1): the corrections that satisfy H e = s (checked on the
    CPU from the sparse H) are exactly the converged shots, and 64 sampled
    shots equal the oracle's bit for bit."""
    from tests import validity

    prob = codes.dem_problem(2736, 26208)
    syn, _ = sampling.sample_syndromes_sparse(prob, 0xDE3, 200000)
    dec = rb.Decoder.from_problem(prob, **dict(RELAY_DEFAULT, io_layout=1))
    print(f"[parity] two-gross full size: B={len(syn)} variant={dec.info()['variant']}", flush=True)
    out = dec.decode(torch.from_numpy(rb.pack_bits(syn)).cuda())
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    dec.close()
    ok = validity.valid_shots(prob, gpu["corr"], syn)
    np.testing.assert_array_equal(ok, gpu["conv"] == 1)
    assert 0.3 < ok.mean() < 1.0
    idx = np.sort(np.random.default_rng(4).choice(len(syn), 64, replace=False))
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, RELAY_DEFAULT, syn[idx])
    np.testing.assert_array_equal(rb.unpack_bits(gpu["corr"][idx], prob.n), ref["corr"])
    for k in ("conv", "legs", "iters", "weight"):
        np.testing.assert_array_equal(gpu[k][idx], ref[k], err_msg=k)


@pytest.mark.parametrize("anchor", [0, 1])
def test_very_long_rows_and_heavy_columns(rb, anchor):
    """Rows of degree up to 250 (eight 32-position records each), columns of
    degree up to 15 (entries past a slot's first four come from the CSC entry
    table), columns of degree 0 and 1 beside them, per-column priors; both
    anchors, S = 2."""
    rng = np.random.default_rng(33)
    m, n = 120, 1500
    h = np.zeros((m, n), np.uint8)
    for i in range(m):
        d = int(rng.integers(150, 251)) if i % 10 == 0 else int(rng.integers(2, 30))
        h[i, rng.choice(n, d, replace=False)] = 1
    heavy = rng.choice(n, 20, replace=False)
    for j in heavy:
        h[rng.choice(m, int(rng.integers(8, 16)), replace=False), j] = 1
    h[:, rng.choice(np.setdiff1d(np.arange(n), heavy), 30, replace=False)] = 0  # empty columns
    prior = rng.uniform(0.005, 0.08, n)
    prob = codes.problem_from_dense("very_long_rows", h, prior, np.zeros((1, n), np.uint8))
    deg_r, deg_c = h.sum(axis=1), h.sum(axis=0)
    assert deg_r.max() > 224 and deg_c.max() > 8 and (deg_c == 0).any() and (deg_c == 1).any()
    _, syn = sampling.sample_batch(prob, 55 + anchor, 0, 120)
    prm = dict(RELAY_DEFAULT, anchor=anchor, num_legs=6, num_solutions=2)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn, want_llr=True)
    vs = _large_variants(rb, prob)
    assert vs
    for v in vs:
        gpu = gpu_decode(rb, prob, prm, syn, variant=v)
        assert_parity(gpu, ref, syn, prob, f"very long rows, anchor {anchor}, large variant {v}")
