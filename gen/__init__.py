"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *makes inputs*: coupling graphs, fields, inverse-temperature
ladders and seeds.  It holds none of the sampling arithmetic (no random-number
generator of the method, no acceptance rule, no energy bookkeeping), so that the
oracle under ``oracle/`` and the HIP library can both be fed from it without
sharing any of the computation they are compared on.
"""
from .chimera import (  # noqa: F401
    LayeredSystem,
    Workload,
    chimera_template,
    make_chimera_system,
    make_random_system,
    make_workload,
    beta_ladder,
    CONFIGS,
)
