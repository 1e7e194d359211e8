"""Seeded synthetic inputs for the l0 search.

This package only *draws* inputs: primary features, rung<=2 operator-tree
features, a planted target and task partitions.  It contains none of the
least-squares arithmetic of the method, so both the CPU oracle (``oracle/``)
and the GPU library (``paper_2502_20072_amd``) may import it without sharing
any of the computation they are compared on.
"""
from .problems import (  # noqa: F401
    Problem,
    CONFIGS,
    make_problem,
    make_config,
    make_batch_problem,
    make_decoy_problem,
    make_batch_problems,
    tiny_problem,
    integer_problem,
    input_digest,
)
from .screening import (  # noqa: F401
    SCREEN_CONFIGS,
    ScreenWorkload,
    all_pairs,
    make_screen_workload,
    screen_digest,
)
