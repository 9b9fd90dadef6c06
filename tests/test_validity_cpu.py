"""The CPU validity check of packed corrections (tests/validity.py) against
dense GF(2) products and planted errors."""
import numpy as np
import pytest

from paper_2511_21660_amd import relaybp as rb
from tests import validity
from workloads import codes, sampling


def test_matches_dense_product_on_bb72():
    prob = codes.bb_problem("bb72", 0.05)
    rng = np.random.default_rng(3)
    syn = rng.integers(0, 2, (500, prob.m), dtype=np.uint8)
    corr = (rng.random((500, prob.n)) < 0.05).astype(np.uint8)
    corr[:40] = 0
    syn[:20] = 0                                   # e = 0 solves s = 0 exactly
    dense = ((corr.astype(np.int64) @ prob.dense().astype(np.int64).T) % 2 == syn).all(1)
    got = validity.valid_shots(prob, rb.pack_bits(corr), syn, chunk=128)
    np.testing.assert_array_equal(got, dense)
    assert got[:20].all()
    np.testing.assert_array_equal(got[20:40], (syn[20:40] == 0).all(1))  # e = 0: valid iff s = 0


def test_faults_are_valid_and_a_flip_is_not():
    dem = codes.dem_problem()
    syn, (fs, fc) = sampling.sample_syndromes_sparse(dem, 11, 3000)
    words = np.zeros((3000, (dem.n + 31) // 32), np.uint32)
    np.bitwise_or.at(words, (fs, fc // 32), np.uint32(1) << (fc % 32).astype(np.uint32))
    assert validity.valid_shots(dem, words, syn, chunk=1000).all()
    j = int(np.nonzero(np.bincount(dem.cols, minlength=dem.n))[0][5])   # a column with checks
    words[7, j // 32] ^= np.uint32(1) << np.uint32(j % 32)
    ok = validity.valid_shots(dem, words, syn, chunk=1000)
    assert not ok[7] and ok[np.arange(3000) != 7].all()
    words[9, -1] |= np.uint32(1) << np.uint32(31)                     # past column N - 1
    with pytest.raises(AssertionError):
        validity.valid_shots(dem, words, syn)
