"""CPU oracle for Relay-BP decoding (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
``paper_2511_21660_amd`` and never imports it.
"""
from .oracle import (  # noqa: F401
    OracleParams,
    build,
    decode,
    decode_windowed,
    gamma_f32,
    lib,
    minsum_trace,
    philox4x32_10,
    round_h16,
    sumproduct_trace,
    tangent,
    trace,
)
