"""GPU parity of the binary16 decoder (rb_params.precision = RB_PREC_F16)
against the oracle's binary16 mode, bit for bit: corrections, converged
flags, legs, iterations, weights and the final marginals (binary16 values
returned as float).

The binary16 kernel decodes two syndromes per workgroup, one in each half of
every packed word, each half running its own legs and shots; the batches
below mix long and short shots so that one half's events happen while the
other half iterates, and odd batch sizes leave a half without a shot."""
import numpy as np
import pytest

import oracle
from tests.conftest import RELAY_DEFAULT
from tests.test_gpu_parity import _irregular_problem, assert_parity
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


def h16_decode(rb, prob, params, syn, variant=None, bits=False, gamma1=None):
    dec = rb.Decoder.from_problem(prob, **dict(params, precision=1, io_layout=1 if bits else 0))
    if variant is not None:
        dec.set_variant(variant)
    if gamma1 is not None:
        dec.set_leg_gamma(1, gamma1)
    d_syn = torch.from_numpy(rb.pack_bits(syn) if bits else np.ascontiguousarray(syn)).cuda()
    out = dec.decode(d_syn, want_llr=True)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if bits:
        res["corr"] = rb.unpack_bits(res["corr"], prob.n)
    res["info"] = dec.info()
    dec.close()
    return res


def h16_ref(prob, params, syn, gamma1=None):
    return oracle.decode(prob.m, prob.n, prob.rows, prob.cols, prob.prior, params, syn, want_llr=True,
                         precision="h16", gamma1=gamma1)


def test_dem_h16_parity(rb, dem):
    """936 x 8785 DEM, R = 20, S = 1: 301 shots (an odd batch)."""
    _, syn = sampling.sample_batch(dem, 41 << 32, 0, 301)
    gpu = h16_decode(rb, dem, RELAY_DEFAULT, syn)
    assert gpu["info"]["threads_per_block"] == 1024
    assert_parity(gpu, h16_ref(dem, RELAY_DEFAULT, syn), syn, dem, "dem h16")


def test_dem_h16_prior_anchor_solutions_cutoff_bits(rb, dem):
    _, syn = sampling.sample_batch(dem, 43 << 32, 0, 160)
    prm = dict(RELAY_DEFAULT, anchor=1, num_solutions=3, num_legs=8, max_total_iters=300)
    gpu = h16_decode(rb, dem, prm, syn, bits=True)
    assert_parity(gpu, h16_ref(dem, prm, syn), syn, dem, "dem h16 prior anchor S=3 cutoff bits")


def test_dem_h16_trace(rb, dem):
    """Message-level hook: 30 iterations of one leg with per-column gamma,
    every marginal equal to the oracle's binary16 trace (4 shots, 2 blocks)."""
    _, syn = sampling.sample_batch(dem, 17, 0, 4)
    gamma = np.random.default_rng(9).uniform(-0.24, 0.66, dem.n).astype(np.float32)
    dec = rb.Decoder.from_problem(dem, **dict(RELAY_DEFAULT, precision=1))
    got = dec.trace(torch.from_numpy(syn).cuda(), torch.from_numpy(gamma).cuda(), 30)
    torch.cuda.synchronize()
    ref = oracle.trace(dem.m, dem.n, dem.rows, dem.cols, dem.prior, gamma, 30, syn, precision="h16")
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    dec.close()


def test_h16_every_block_shape_irregular_and_bb(rb):
    """Irregular graphs (empty rows and columns, a degree-1 check, erasures)
    and [[144,12,12]] on every block shape that fits, both anchors."""
    for prob, key in ((_irregular_problem(3), 77), (_irregular_problem(4), 79),
                      (codes.bb_problem("bb144", 0.06), 81)):
        _, syn = sampling.sample_batch(prob, key, 0, 201)
        syn[:3] = 1
        d = rb.Decoder.from_problem(prob, **dict(RELAY_DEFAULT, precision=1))
        nvar = d.info()["num_variants"]
        d.close()
        tested = 0
        for anchor in (0, 1):
            prm = dict(RELAY_DEFAULT, anchor=anchor, num_solutions=2, num_legs=10)
            ref = h16_ref(prob, prm, syn)
            for v in range(nvar):
                try:
                    gpu = h16_decode(rb, prob, prm, syn, variant=v)
                except rb.RelayError as e:
                    assert e.status == 8
                    continue
                assert_parity(gpu, ref, syn, prob, f"h16 {prob.name} anchor={anchor} variant={v}")
                tested += 1
        assert tested >= 4


def test_h16_long_rows_split_over_two_lanes(rb):
    """Rows of degree 33..90 split over lane pairs, which merge their minima
    and parities; uniform priors make every |nu| tie at the first iteration."""
    rng = np.random.default_rng(11)
    m, n = 60, 700
    h = np.zeros((m, n), np.uint8)
    for i in range(m):
        deg = int(rng.integers(33, 91)) if i % 3 == 0 else int(rng.integers(2, 12))
        h[i, rng.choice(n, deg, replace=False)] = 1
    h[:, h.sum(0) > 6] = 0
    h[:, h.sum(0) == 0] = 0
    prob = codes.problem_from_dense("longrows", h, 0.02, np.zeros((1, n), np.uint8))
    _, syn = sampling.sample_batch(prob, 5, 0, 151)
    assert_parity(h16_decode(rb, prob, RELAY_DEFAULT, syn), h16_ref(prob, RELAY_DEFAULT, syn), syn, prob,
                  "h16 long rows")


def test_h16_learned_first_leg(rb):
    prob = codes.bb_problem("bb144", 0.05)
    _, syn = sampling.sample_batch(prob, 83, 0, 120)
    g1 = np.random.default_rng(3).uniform(-0.2, 0.6, prob.n).astype(np.float32)
    prm = dict(RELAY_DEFAULT, num_legs=6)
    assert_parity(h16_decode(rb, prob, prm, syn, gamma1=g1), h16_ref(prob, prm, syn, gamma1=g1), syn, prob,
                  "h16 learned leg")


def test_h16_small_and_empty_batches(rb, dem):
    _, syn = sampling.sample_batch(dem, 47 << 32, 0, 3)
    for b in (1, 2, 3):
        assert_parity(h16_decode(rb, dem, RELAY_DEFAULT, syn[:b]), h16_ref(dem, RELAY_DEFAULT, syn[:b]), syn[:b],
                      dem, f"h16 B={b}")
    dec = rb.Decoder.from_problem(dem, **dict(RELAY_DEFAULT, precision=1))
    out = dec.decode(torch.zeros((0, dem.m), dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert out["corr"].shape == (0, dem.n)
    dec.close()


def test_h16_unsupported_calls(rb):
    prob = codes.bb_problem("bb72", 0.05)
    dec = rb.Decoder.from_problem(prob, **dict(RELAY_DEFAULT, precision=1))
    with pytest.raises(rb.RelayError) as e:
        dec.set_prior_scale(0.5)
    assert e.value.status == 8
    with pytest.raises(rb.RelayError) as e:
        rb.MultiDecoder([prob, prob], **dict(RELAY_DEFAULT, precision=1))
    assert e.value.status == 8
    dec.close()
