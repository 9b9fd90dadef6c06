import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Relay parameters of the paper's appendix on Relay resources (T = 80 for the
# first leg, 60 after, gamma_0 = 0.125, gamma ~ U[-0.24, 0.66] for later legs),
# with R legs in total and S solutions.
RELAY_DEFAULT = dict(num_legs=20, iters_first=80, iters_leg=60, num_solutions=1,
                     gamma_first=0.125, gamma_lo=-0.24, gamma_hi=0.66,
                     llr_clip=2.0 ** 64, seed=0x52454C4159, anchor=0, max_total_iters=0)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def relay_default():
    return dict(RELAY_DEFAULT)


def logical_failures_np(prob, faults, corr, conv):
    """Per-shot logical failure: not converged, or the residual F + F_hat
    anticommutes with a row of the logical matrix."""
    import numpy as np

    resid = (faults ^ corr).astype(np.int64)
    bad = ((prob.logical.astype(np.int64) @ resid.T) % 2).any(0)
    return (~conv.astype(bool)) | bad
