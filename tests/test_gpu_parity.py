"""GPU parity: the HIP decoder against the CPU oracle on identical seeded inputs.

Both sides run the same canonical FP32 operation order, so the bar is
bit-exact for corrections, converged flags, leg and iteration counts and
weights, and for the FP32 marginals (which bounds the relative error of the
messages at 0, inside the 1e-5 tolerance the decoder is specified to).
"""
import numpy as np
import pytest

import oracle
from tests.conftest import RELAY_DEFAULT
from workloads import codes, sampling

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("corr", "conv", "legs", "iters", "weight", "llr")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2511_21660_amd import relaybp

    relaybp.load_library()
    return relaybp


def gpu_decode(rb, prob, params, syn, variant=None):
    dec = rb.Decoder.from_problem(prob, **params)
    if variant is not None:
        dec.set_variant(variant)
    out = dec.decode(torch.from_numpy(np.ascontiguousarray(syn)).cuda(), want_llr=True)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["info"] = dec.info()
    dec.close()
    return res


def assert_parity(gpu, ref, syn, prob, label):
    print(f"[parity] {label}: B={len(syn)} variant={gpu['info']['variant']}", flush=True)
    for k in KEYS:
        g, r = gpu[k], ref[k]
        if not np.array_equal(g, r):
            rows = np.nonzero((g != r).reshape(len(syn), -1).any(1))[0]
            raise AssertionError(f"{label}: '{k}' differs on {rows.size} shots, first {rows[:8]}")
    h = prob.dense().astype(np.int64)
    ok = (gpu["corr"].astype(np.int64) @ h.T) % 2 == (syn != 0)
    assert ok[gpu["conv"] == 1].all()


def test_gamma_table_bit_exact(rb):
    prob = codes.bb_problem("bb144", 0.04)
    prm = dict(RELAY_DEFAULT, num_legs=301)
    dec = rb.Decoder.from_problem(prob, **prm)
    tab = dec.gamma_table()
    assert tab.shape == (301, 144)
    assert (tab[0] == np.float32(0.125)).all()
    for r in (2, 3, 17, 301):
        for j in range(144):
            assert tab[r - 1, j] == oracle.gamma_f32(prm["seed"], r, j, prm["gamma_lo"],
                                                      prm["gamma_hi"])


def test_trace_messages_bit_exact(rb):
    """One leg, per-column gamma, 40 iterations with no early stop: every
    marginal Lambda_j(t) equal to the oracle's."""
    prob = codes.bb_problem("bb72", 0.05)
    _, syn = sampling.sample_batch(prob, 11, 0, 96)
    rng = np.random.default_rng(3)
    gamma = rng.uniform(-0.24, 0.66, prob.n).astype(np.float32)
    dec = rb.Decoder.from_problem(prob, **RELAY_DEFAULT)
    for scale in (1.0, 0.75):
        tr = dec.trace(torch.from_numpy(syn).cuda(), torch.from_numpy(gamma).cuda(), 40,
                       scale=scale).cpu().numpy()
        ref = oracle.trace(prob.m, prob.n, prob.rows, prob.cols, prob.prior, gamma, 40, syn,
                           scale=scale)
        np.testing.assert_array_equal(tr, ref)


def test_cfg1_bb72_full_parity(rb):
    """[[72,12,6]], p = 0.05, 1000 shots, T = 80/60, R = 20, S = 1."""
    prob = codes.bb_problem("bb72", 0.05)
    _, syn = sampling.sample_batch(prob, (1 << 32) | 0, 0, 1000)
    gpu = gpu_decode(rb, prob, RELAY_DEFAULT, syn)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, RELAY_DEFAULT, syn,
                        want_llr=True)
    assert_parity(gpu, ref, syn, prob, "cfg1")


@pytest.mark.parametrize("p", [0.02, 0.04, 0.06, 0.08])
def test_cfg2_bb144_subset_parity(rb, p):
    """[[144,12,12]], R = 301, S = 5: 600 shots per p (several slots per wave,
    a ragged last wave, and long failing shots)."""
    prob = codes.bb_problem("bb144", p)
    q = [0.02, 0.04, 0.06, 0.08].index(p)
    _, syn = sampling.sample_batch(prob, (2 << 32) | q, 0, 600)
    prm = dict(RELAY_DEFAULT, num_legs=301, num_solutions=5)
    gpu = gpu_decode(rb, prob, prm, syn)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn,
                        want_llr=True)
    assert_parity(gpu, ref, syn, prob, f"cfg2 p={p}")


@pytest.mark.parametrize("name", ["bb90", "bb288"])
def test_other_bb_codes_parity(rb, name):
    prob = codes.bb_problem(name, 0.04)
    _, syn = sampling.sample_batch(prob, 4 << 32, 0, 500)
    gpu = gpu_decode(rb, prob, RELAY_DEFAULT, syn)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, RELAY_DEFAULT, syn,
                        want_llr=True)
    assert_parity(gpu, ref, syn, prob, name)


def test_every_fitting_variant_agrees(rb):
    """Results do not depend on the kernel configuration (tile, lanes per shot, grid)."""
    prob = codes.bb_problem("bb144", 0.06)
    _, syn = sampling.sample_batch(prob, 99, 0, 400)
    prm = dict(RELAY_DEFAULT, num_legs=60, num_solutions=2)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn,
                        want_llr=True)
    nvar = gpu_decode(rb, prob, prm, syn[:1])["info"]["num_variants"]
    tested = 0
    for v in range(nvar):
        try:
            gpu = gpu_decode(rb, prob, prm, syn, variant=v)
        except rb.RelayError as e:
            assert e.status == 8
            continue
        assert_parity(gpu, ref, syn, prob, f"variant {v}")
        tested += 1
    assert tested >= 3


def test_every_fitting_variant_nonuniform_priors(rb):
    """A BB graph with a different prior on every column (the kernels' general
    solution-weight path; uniform priors take a count x w path): every
    fitting configuration against the oracle, two solutions per shot."""
    base = codes.bb_problem("bb144", 0.05)
    rng = np.random.default_rng(31)
    prior = rng.uniform(0.02, 0.09, base.n)
    prob = codes.problem_from_dense("bb144-nonuniform", base.dense(), prior, base.logical)
    faults = (rng.random((300, prob.n)) < prior[None, :]).astype(np.uint8)
    syn = ((faults.astype(np.int64) @ base.dense().T.astype(np.int64)) % 2).astype(np.uint8)
    prm = dict(RELAY_DEFAULT, num_legs=40, num_solutions=2)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn, want_llr=True)
    nvar = gpu_decode(rb, prob, prm, syn[:1])["info"]["num_variants"]
    tested = 0
    for v in range(nvar):
        try:
            gpu = gpu_decode(rb, prob, prm, syn, variant=v)
        except rb.RelayError as e:
            assert e.status == 8
            continue
        assert_parity(gpu, ref, syn, prob, f"non-uniform priors variant {v}")
        tested += 1
    assert tested >= 3


def _irregular_problem(seed, m=40, n=90):
    rng = np.random.default_rng(seed)
    h = (rng.random((m, n)) < 0.06).astype(np.uint8)
    h[rng.integers(0, m), :] = 0           # an empty row
    h[:, rng.integers(0, n)] = 0           # an empty column
    r1 = rng.integers(0, m)
    h[r1, :] = 0
    h[r1, rng.integers(0, n)] = 1          # a degree-1 check
    h = h[:, :n]
    h[:, h.sum(0) > 8] = 0
    h[h.sum(1) > 16, :] = 0
    prior = rng.uniform(0.01, 0.2, n)
    prior[rng.integers(0, n, 3)] = 0.5     # erasures: w = 0
    prob = codes.problem_from_dense(f"irr{seed}", h, prior, np.zeros((1, n), np.uint8))
    return prob


@pytest.mark.parametrize("anchor", [0, 1])
@pytest.mark.parametrize("seed", [1, 2])
def test_irregular_graph_edge_cases(rb, seed, anchor):
    """Empty rows (unsatisfiable when their syndrome bit is 1), empty columns,
    degree-1 checks (saturated messages), erasure priors (w = 0), both
    anchors, S = 3, and an iteration cutoff."""
    prob = _irregular_problem(seed)
    _, syn = sampling.sample_batch(prob, 5 + seed, 0, 300)
    syn[:5] = 0
    syn[5:10] = 1
    for prm in (dict(RELAY_DEFAULT, anchor=anchor, num_solutions=3, num_legs=12),
                dict(RELAY_DEFAULT, anchor=anchor, num_legs=40, max_total_iters=250)):
        gpu = gpu_decode(rb, prob, prm, syn)
        ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn,
                            want_llr=True)
        assert_parity(gpu, ref, syn, prob, f"irregular seed={seed} anchor={anchor}")


def test_irregular_graph_every_variant(rb):
    """Irregular graph (empty rows and columns, a degree-1 check, erasures) on
    every kernel configuration that fits it, group tiles and block shapes."""
    prob = _irregular_problem(3)
    _, syn = sampling.sample_batch(prob, 77, 0, 250)
    syn[:4] = 1
    prm = dict(RELAY_DEFAULT, num_solutions=2, num_legs=10)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn,
                        want_llr=True)
    nvar = gpu_decode(rb, prob, prm, syn[:1])["info"]["num_variants"]
    tested = []
    for v in range(nvar):
        try:
            gpu = gpu_decode(rb, prob, prm, syn, variant=v)
        except rb.RelayError as e:
            assert e.status == 8
            continue
        assert_parity(gpu, ref, syn, prob, f"variant {v}")
        tested.append(gpu["info"]["threads_per_block"])
    assert len(tested) >= 3 and max(tested) >= 512  # block shapes included


def test_long_rows_split_over_two_lanes(rb):
    """Rows longer than 32 are split over two lanes of the block kernel, which
    merge min1/min2, the minimum's position and the parities.  Uniform priors
    make every |nu| equal at the first iteration, so ties between the two
    halves occur; rows of degree 33..90 and short rows side by side."""
    rng = np.random.default_rng(11)
    m, n = 24, 400
    h = np.zeros((m, n), np.uint8)
    for i, d in enumerate([90, 77, 64, 50, 41, 33] + [int(x) for x in rng.integers(3, 12, m - 6)]):
        h[i, rng.choice(n, d, replace=False)] = 1
    prior = np.full(n, 0.05)
    prob = codes.problem_from_dense("long_rows", h, prior, np.zeros((1, n), np.uint8))
    _, syn = sampling.sample_batch(prob, 1234, 0, 300)
    prm = dict(RELAY_DEFAULT, num_legs=6, num_solutions=2)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn, want_llr=True)
    gpu = gpu_decode(rb, prob, prm, syn)
    assert gpu["info"]["threads_per_block"] >= 512
    assert_parity(gpu, ref, syn, prob, "long rows")


@pytest.mark.parametrize("name,anchor", [("bb144", 0), ("bb144", 1), ("dem", 0), ("dem-large", 0),
                                         ("dem-large", 1)])
def test_learned_first_leg_parity(rb, name, anchor):
    """rb_set_leg_gamma / rb_set_prior_scale (a learned first leg inside Relay)
    against the oracle's gamma1 / scale, on the group kernel ([[144,12,12]]),
    the block kernel (DEM-shaped matrix) and the large-graph kernel chosen
    before the setters run (its gamma table by fault slot must follow them);
    the table readback shows the row."""
    prob = codes.dem_problem() if name.startswith("dem") else codes.bb_problem(name, 0.05)
    _, syn = sampling.sample_batch(prob, 71, 0, 120 if name.startswith("dem") else 400)
    g1 = np.random.default_rng(8).uniform(-0.2, 0.6, prob.n).astype(np.float32)
    prm = dict(RELAY_DEFAULT, anchor=anchor, num_legs=6, num_solutions=2)
    dec = rb.Decoder.from_problem(prob, **prm)
    if name == "dem-large":
        large = []
        for v in range(dec.info()["num_variants"]):
            try:
                if rb.plan_check(prob.m, prob.n, prob.rows, prob.cols, v)["block_kernel"] == 2:
                    large.append(v)
            except rb.RelayError as e:
                assert e.status == 8
        assert large
        dec.set_variant(large[0])
    dec.set_leg_gamma(1, g1)
    dec.set_prior_scale(0.8)
    np.testing.assert_array_equal(dec.gamma_table()[0], g1)
    out = dec.decode(torch.from_numpy(syn).cuda(), want_llr=True)
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    gpu["info"] = dec.info()
    dec.close()
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn, want_llr=True,
                        gamma1=g1, scale=0.8)
    assert_parity(gpu, ref, syn, prob, f"learned first leg {name} anchor {anchor}")


@pytest.mark.parametrize("scale", [0.0, -1.0])
def test_signed_zero_channel_llrs(rb, scale):
    """Channel LLRs s * w that are -0 (s = 0 with priors above 1/2, s = -1 with
    priors of exactly 1/2) on every configuration that fits, both anchors:
    the kernels take such a zero as +0 when a syndrome starts (the group
    kernel reads signs as sign bits), which must leave every output equal to
    the oracle's, whose sign test is x < 0."""
    prob = _irregular_problem(23)
    prior = prob.prior.copy()
    rng = np.random.default_rng(5)
    prior[rng.integers(0, prob.n, 8)] = 0.5
    prior[rng.integers(0, prob.n, 8)] = 0.7
    prob = codes.problem_from_dense("irr23-zeros", prob.dense(), prior, prob.logical)
    _, syn = sampling.sample_batch(prob, 41, 0, 200)
    for anchor in (0, 1):
        prm = dict(RELAY_DEFAULT, anchor=anchor, num_legs=8, num_solutions=2)
        ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn, want_llr=True,
                            scale=scale)
        probe = rb.Decoder.from_problem(prob, **prm)
        nvar = probe.info()["num_variants"]
        probe.close()
        tested = 0
        for v in range(nvar):
            dec = rb.Decoder.from_problem(prob, **prm)
            try:
                dec.set_variant(v)
            except rb.RelayError as e:
                assert e.status == 8
                dec.close()
                continue
            dec.set_prior_scale(scale)
            out = dec.decode(torch.from_numpy(syn).cuda(), want_llr=True)
            torch.cuda.synchronize()
            gpu = {k: x.cpu().numpy() for k, x in out.items()}
            gpu["info"] = dec.info()
            dec.close()
            assert_parity(gpu, ref, syn, prob, f"scale {scale} anchor {anchor} variant {v}")
            tested += 1
        assert tested >= 3


def test_unsatisfiable_syndrome_runs_full_budget(rb):
    code = codes.bb_code("bb72")
    h = np.vstack([code.hx, np.zeros((1, 72), np.uint8)])
    prob = codes.problem_from_dense("bb72+empty", h, 0.04, code.logical)
    syn = np.zeros((3, 37), np.uint8)
    syn[:, 36] = 1
    syn[1, 0] = 1
    prm = dict(RELAY_DEFAULT, num_legs=301)
    gpu = gpu_decode(rb, prob, prm, syn)
    assert (gpu["iters"] == 18080).all() and (gpu["legs"] == 301).all()
    assert (gpu["conv"] == 0).all()
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn,
                        want_llr=True)
    assert_parity(gpu, ref, syn, prob, "unsatisfiable")


def test_empty_and_single_batches(rb):
    prob = codes.bb_problem("bb72", 0.05)
    dec = rb.Decoder.from_problem(prob, **RELAY_DEFAULT)
    out = dec.decode(torch.zeros((0, prob.m), dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert out["corr"].shape == (0, prob.n)
    syn = np.zeros((1, prob.m), np.uint8)
    out = dec.decode(torch.from_numpy(syn).cuda())
    torch.cuda.synchronize()
    assert out["conv"].item() == 1 and out["iters"].item() == 1 and out["corr"].sum().item() == 0


def test_batch_order_invariance(rb):
    prob = codes.bb_problem("bb144", 0.07)
    _, syn = sampling.sample_batch(prob, 123, 0, 700)
    prm = dict(RELAY_DEFAULT, num_legs=40)
    a = gpu_decode(rb, prob, prm, syn)
    perm = np.random.default_rng(1).permutation(len(syn))
    b = gpu_decode(rb, prob, prm, syn[perm])
    for k in KEYS:
        np.testing.assert_array_equal(a[k][perm], b[k])


def test_cfg2_full_size_sampled_parity(rb):
    """The benchmark's workload at full size (10^5 shots at p = 0.08, R = 301,
    S = 5, the launch configuration the benchmark times): every converged
    correction valid, and 400 sampled shots bit-exact against the oracle."""
    prob = codes.bb_problem("bb144", 0.08)
    _, syn = sampling.sample_batch(prob, (2 << 32) | 3, 0, 100000)
    prm = dict(RELAY_DEFAULT, num_legs=301, num_solutions=5)
    gpu = gpu_decode(rb, prob, prm, syn)
    h = prob.dense().astype(np.int64)
    ok = (gpu["corr"].astype(np.int64) @ h.T) % 2 == syn
    assert ok[gpu["conv"] == 1].all()
    idx = np.random.default_rng(0).choice(len(syn), 400, replace=False)
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn[idx],
                        want_llr=True)
    sub = {k: gpu[k][idx] for k in KEYS}
    sub["info"] = gpu["info"]
    assert_parity(sub, ref, syn[idx], prob, "cfg2 full-size sample")


@pytest.fixture(scope="module")
def dem():
    return codes.dem_problem()


def test_dem_block_kernel_parity(rb, dem):
    """DEM-shaped 936 x 8785 matrix (E = 27,617, row degree up to 63): the
    block kernel against the oracle on 2000 shots (over the first 1000 one per
    CU, so each slot of the persistent queue runs several shots), T = 80/60,
    R = 20, S = 1."""
    _, syn = sampling.sample_batch(dem, 3 << 32, 0, 2000)
    gpu = gpu_decode(rb, dem, RELAY_DEFAULT, syn)
    assert gpu["info"]["threads_per_block"] >= 512
    ref = oracle.decode(dem.m, dem.n, dem.rows, dem.cols, dem.prior, RELAY_DEFAULT, syn,
                        want_llr=True)
    assert_parity(gpu, ref, syn, dem, "dem block")


def test_dem_full_size_validity_and_sampled_parity(rb, dem):
    """The DEM-shaped 936 x 8785 workload at full size, in the launch
    configuration the benchmark times (the same 10^6 seeded syndromes,
    bit-packed in and out, R = 20, S = 1, the default configuration): the
    corrections that satisfy H e = s (checked on the CPU from the sparse H)
    are exactly the converged shots, and 1000 sampled shots equal the
    oracle's bit for bit."""
    from tests import validity

    syn, _ = sampling.sample_syndromes_sparse(dem, 0xDE3, 10 ** 6)
    dec = rb.Decoder.from_problem(dem, **dict(RELAY_DEFAULT, io_layout=1))
    print(f"[parity] dem full size: B={len(syn)} variant={dec.info()['variant']}", flush=True)
    out = dec.decode(torch.from_numpy(rb.pack_bits(syn)).cuda())
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    dec.close()
    ok = validity.valid_shots(dem, gpu["corr"], syn)
    np.testing.assert_array_equal(ok, gpu["conv"] == 1)
    assert 0.9 < ok.mean() < 1.0
    idx = np.sort(np.random.default_rng(1).choice(len(syn), 1000, replace=False))
    ref = oracle.decode(dem.m, dem.n, dem.rows, dem.cols, dem.prior, RELAY_DEFAULT, syn[idx])
    np.testing.assert_array_equal(rb.unpack_bits(gpu["corr"][idx], dem.n), ref["corr"])
    for k in ("conv", "legs", "iters", "weight"):
        np.testing.assert_array_equal(gpu[k][idx], ref[k], err_msg=k)


def test_dem_trace_bit_exact(rb, dem):
    _, syn = sampling.sample_batch(dem, 17, 0, 4)
    gamma = np.random.default_rng(9).uniform(-0.24, 0.66, dem.n).astype(np.float32)
    dec = rb.Decoder.from_problem(dem, **RELAY_DEFAULT)
    tr = dec.trace(torch.from_numpy(syn).cuda(), torch.from_numpy(gamma).cuda(), 25).cpu().numpy()
    ref = oracle.trace(dem.m, dem.n, dem.rows, dem.cols, dem.prior, gamma, 25, syn)
    np.testing.assert_array_equal(tr, ref)


def test_dem_prior_anchor_and_solutions(rb, dem):
    _, syn = sampling.sample_batch(dem, 5 << 32, 0, 120)
    prm = dict(RELAY_DEFAULT, anchor=1, num_solutions=3, num_legs=8, max_total_iters=300)
    gpu = gpu_decode(rb, dem, prm, syn)
    ref = oracle.decode(dem.m, dem.n, dem.rows, dem.cols, dem.prior, prm, syn, want_llr=True)
    assert_parity(gpu, ref, syn, dem, "dem prior anchor S=3")


# ----------------------------------------------------------- mixed batches

MIX_CODES = ("bb72", "bb90", "bb144", "bb288")
MIX_PATTERN = np.array([0, 1, 2, 0, 3, 1, 0, 2, 1, 0], np.int32)  # 4:3:2:1 interleave


def _mixed_inputs(b, p=0.04, key=4 << 32):
    probs = [codes.bb_problem(n, p) for n in MIX_CODES]
    code_id = np.resize(MIX_PATTERN, b).astype(np.int32)
    m_max = max(pr.m for pr in probs)
    syn = np.zeros((b, m_max), np.uint8)
    per_code = {}
    for k, pr in enumerate(probs):
        idx = np.nonzero(code_id == k)[0]
        _, s = sampling.sample_batch(pr, key | k, 0, idx.size)
        syn[idx, :pr.m] = s
        per_code[k] = (idx, s)
    return probs, code_id, syn, per_code


def test_mixed_batch_parity(rb):
    """Four BB codes interleaved 4:3:2:1 in one launch: every shot equals the
    oracle's decode of its own code."""
    b = 1200
    probs, code_id, syn, per_code = _mixed_inputs(b)
    dec = rb.MultiDecoder(probs, **RELAY_DEFAULT)
    out = dec.decode(torch.from_numpy(code_id).cuda(), torch.from_numpy(syn).cuda(), want_llr=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if k != "workspace"}
    for k, pr in enumerate(probs):
        idx, s = per_code[k]
        ref = oracle.decode(pr.m, pr.n, pr.rows, pr.cols, pr.prior, RELAY_DEFAULT, s, want_llr=True)
        sub = {"corr": g["corr"][idx, :pr.n], "conv": g["conv"][idx], "legs": g["legs"][idx],
               "iters": g["iters"][idx], "weight": g["weight"][idx], "llr": g["llr"][idx, :pr.n],
               "info": {"variant": "mixed"}}
        assert_parity(sub, ref, s, pr, f"mixed code {MIX_CODES[k]}")
    dec.close()


def test_mixed_full_size_parity(rb):
    """The mixed-codes workload at full size, in the launch configuration the
    benchmark times: the same 4x10^5 seeded syndromes of four BB codes
    (4:3:2:1, p = 0.04, R = 20), tiles chosen by the autotuner on the first
    20000 syndromes of each code, one mixed launch; every shot equals the
    oracle's decode of its own code."""
    b = 400000
    probs, code_id, syn, per_code = _mixed_inputs(b)
    dec = rb.MultiDecoder(probs, **RELAY_DEFAULT)
    chosen = dec.autotune([torch.from_numpy(per_code[k][1][:20000]).cuda() for k in range(len(probs))], reps=2)
    print(f"[parity] mixed full size: B={b} tiles={chosen}", flush=True)
    out = dec.decode(torch.from_numpy(code_id).cuda(), torch.from_numpy(syn).cuda())
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if k != "workspace"}
    dec.close()
    for k, pr in enumerate(probs):
        idx, s = per_code[k]
        ref = oracle.decode(pr.m, pr.n, pr.rows, pr.cols, pr.prior, RELAY_DEFAULT, s)
        np.testing.assert_array_equal(g["corr"][idx, :pr.n], ref["corr"], err_msg=MIX_CODES[k])
        for key in ("conv", "legs", "iters", "weight"):
            np.testing.assert_array_equal(g[key][idx], ref[key], err_msg=f"{MIX_CODES[k]} {key}")
        ok = (ref["corr"].astype(np.int64) @ pr.dense().astype(np.int64).T) % 2 == s
        np.testing.assert_array_equal(ok.all(1), ref["conv"] == 1)


def test_mixed_batch_every_tile(rb):
    """Every tile of the mixed kernel that fits a code, forced per code
    (rb_set_code_variant), in rounds that give each code its next fitting
    tile: every shot equals the oracle's decode of its own code."""
    b = 700
    probs, code_id, syn, per_code = _mixed_inputs(b, p=0.05, key=11 << 32)
    dec = rb.MultiDecoder(probs, **RELAY_DEFAULT)
    nvar = rb.Decoder.from_problem(probs[0], **RELAY_DEFAULT).info()["num_variants"]
    fits = []
    for k in range(len(probs)):
        ok = []
        for v in range(nvar):
            try:
                dec.set_code_variant(k, v)
            except rb.RelayError as e:
                assert e.status == 8  # RB_E_UNSUPPORTED
                continue
            ok.append(v)
        assert ok, MIX_CODES[k]
        fits.append(ok)
    assert any(max(ok) >= 11 for ok in fits)  # the one-syndrome-per-wave tiles take part
    refs = [oracle.decode(pr.m, pr.n, pr.rows, pr.cols, pr.prior, RELAY_DEFAULT, per_code[k][1], want_llr=True)
            for k, pr in enumerate(probs)]
    d_code, d_syn = torch.from_numpy(code_id).cuda(), torch.from_numpy(syn).cuda()
    for rnd in range(max(len(ok) for ok in fits)):
        tiles = [ok[rnd % len(ok)] for ok in fits]
        for k, v in enumerate(tiles):
            dec.set_code_variant(k, v)
        print(f"[parity] mixed tiles {tiles}", flush=True)
        out = dec.decode(d_code, d_syn, want_llr=True)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items() if k != "workspace"}
        for k, pr in enumerate(probs):
            idx, s = per_code[k]
            sub = {"corr": g["corr"][idx, :pr.n], "conv": g["conv"][idx], "legs": g["legs"][idx],
                   "iters": g["iters"][idx], "weight": g["weight"][idx], "llr": g["llr"][idx, :pr.n],
                   "info": {"variant": f"mixed tile {tiles[k]}"}}
            assert_parity(sub, refs[k], s, pr, f"mixed code {MIX_CODES[k]} tile {tiles[k]}")
    dec.close()


def _defined(out, code_id, ns):
    """Outputs with the padding of each row (entries >= N of its code) zeroed."""
    cid = torch.as_tensor(code_id, device="cuda").long()
    n_of = torch.as_tensor(ns, device="cuda")[cid]
    res = {}
    for k, v in out.items():
        if k == "workspace":
            continue
        if v.dim() == 2:
            mask = torch.arange(v.shape[1], device="cuda")[None, :] < n_of[:, None]
            v = torch.where(mask, v, torch.zeros_like(v))
        res[k] = v.clone()
    return res


def test_mixed_autotune_keeps_results(rb):
    b = 600
    probs, code_id, syn, per_code = _mixed_inputs(b, key=7 << 32)
    dec = rb.MultiDecoder(probs, **RELAY_DEFAULT)
    d_code, d_syn = torch.from_numpy(code_id).cuda(), torch.from_numpy(syn).cuda()
    ns = [pr.n for pr in probs]
    before = _defined(dec.decode(d_code, d_syn, want_llr=True), code_id, ns)
    samples = [torch.from_numpy(per_code[k][1]).cuda() for k in range(len(probs))]
    chosen = dec.autotune(samples, reps=1)
    assert len(chosen) == len(probs)
    after = _defined(dec.decode(d_code, d_syn, want_llr=True), code_id, ns)
    torch.cuda.synchronize()
    for k in before:
        assert torch.equal(before[k], after[k]), k


def test_mixed_hipgraph_replays(rb):
    """rb_decode_multi captured in a hipGraph (through torch.cuda.CUDAGraph) and
    replayed several times, with eager work and synchronisation in between:
    every replay equals the eager result."""
    b = 800
    probs, code_id, syn, _ = _mixed_inputs(b, key=9 << 32)
    dec = rb.MultiDecoder(probs, **RELAY_DEFAULT)
    d_code, d_syn = torch.from_numpy(code_id).cuda(), torch.from_numpy(syn).cuda()
    ns = [pr.n for pr in probs]
    eager = _defined(dec.decode(d_code, d_syn), code_id, ns)
    torch.cuda.synchronize()
    out = dec.alloc(b)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        dec.decode(d_code, d_syn, out=out)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        dec.decode(d_code, d_syn, out=out)
    for rep in range(3):
        for v in out.values():
            v.fill_(0x5A if v.dtype == torch.uint8 else 7)  # poison between replays
        junk = torch.randn(1 << 16, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = _defined(out, code_id, ns)
        for k in eager:
            assert torch.equal(got[k], eager[k]), f"replay {rep}: {k}"
        del junk


def test_longest_first_schedule_keeps_results(rb):
    """rb_reserve switches rb_decode to a shot list sorted by syndrome weight;
    every shot's result is unchanged."""
    prob = codes.bb_problem("bb144", 0.07)
    _, syn = sampling.sample_batch(prob, 31, 0, 3000)
    prm = dict(RELAY_DEFAULT, num_legs=60, num_solutions=2)
    dec = rb.Decoder.from_problem(prob, **prm)
    d_syn = torch.from_numpy(syn).cuda()
    plain = {k: v.cpu().numpy() for k, v in dec.decode(d_syn, want_llr=True).items()}
    dec.reserve(4000)
    lpt = {k: v.cpu().numpy() for k, v in dec.decode(d_syn, want_llr=True).items()}
    for k in plain:
        np.testing.assert_array_equal(plain[k], lpt[k])
    ref = oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, prm, syn[:500],
                        want_llr=True)
    sub = {k: lpt[k][:500] for k in KEYS}
    sub["info"] = dec.info()
    assert_parity(sub, ref, syn[:500], prob, "longest-first")


def test_mixed_family_of_noise_rates(rb):
    """One graph at several noise rates plus a second graph in one launch: the
    codes sharing the graph form one family (one shot list; every slot takes w
    and Gamma from its own shot's code), and every shot still equals the
    oracle's decode of its own code (S = 2, so convergence events, leg
    changes and new shots all read the per-shot code)."""
    specs = [("bb72", 0.03), ("bb72", 0.05), ("bb90", 0.04), ("bb72", 0.07)]
    probs = [codes.bb_problem(nm, p) for nm, p in specs]
    b = 2000
    pattern = np.array([0, 1, 3, 2, 1, 0, 3, 3, 2, 1], np.int32)
    code_id = np.resize(pattern, b).astype(np.int32)
    m_max = max(pr.m for pr in probs)
    syn = np.zeros((b, m_max), np.uint8)
    per = []
    for k, pr in enumerate(probs):
        idx = np.nonzero(code_id == k)[0]
        _, s = sampling.sample_batch(pr, (11 << 32) | k, 0, idx.size)
        syn[idx, :pr.m] = s
        per.append((idx, s))
    prm = dict(RELAY_DEFAULT, num_solutions=2)
    dec = rb.MultiDecoder(probs, **prm)
    out = dec.decode(torch.from_numpy(code_id).cuda(), torch.from_numpy(syn).cuda(), want_llr=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if k != "workspace"}
    for k, pr in enumerate(probs):
        idx, s = per[k]
        ref = oracle.decode(pr.m, pr.n, pr.rows, pr.cols, pr.prior, prm, s, want_llr=True)
        sub = {"corr": g["corr"][idx, :pr.n], "conv": g["conv"][idx], "legs": g["legs"][idx],
               "iters": g["iters"][idx], "weight": g["weight"][idx], "llr": g["llr"][idx, :pr.n],
               "info": {"variant": "mixed family"}}
        assert_parity(sub, ref, s, pr, f"family member {specs[k]}")
    dec.close()
