"""Seeded synthetic inputs for Relay-BP decoding.

This package builds decoding problems (check matrices, fault priors, logical
matrices) and samples faults and syndromes from fixed counter-based keys.  It
holds none of the decoder's arithmetic: both the CPU oracle (``oracle/``) and
the HIP library (``paper_2511_21660_amd``) consume what it produces, and it
imports neither of them.

Decoding-problem model (paper Sec. 2.1): a binary matrix H (M x N), a logical
action matrix A (K x N) and per-fault probabilities p; a fault set F occurs
with probability prod_j (1-p_j) (p_j/(1-p_j))^F_j and yields the syndrome
sigma = H F over GF(2); a correction F_hat succeeds iff A (F + F_hat) = 0.
"""
