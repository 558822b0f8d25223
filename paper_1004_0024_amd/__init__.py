"""MI355X parallel-tempering Metropolis library: Python binding of libising.so.

The binding only marshals arguments: every step of the sampler runs in the
HIP kernels behind the C ABI of ``include/ising.h``.  PyTorch supplies device
memory and the current stream.  Importing works without a GPU; any call that
needs the library raises if ``libising.so`` has not been built.
"""
from .binding import (  # noqa: F401
    ACCEPT_ACCURATE,
    ACCEPT_EXACT,
    ACCEPT_FAST,
    ISING_N_STATS,
    STAT_ATTEMPTS,
    STAT_NEAR,
    STAT_WAVE_FLIP,
    STAT_WAVE_STEPS,
    IsingError,
    Mlp,
    Replay,
    Graph,
    State,
    acceptance_row,
    lib,
    lib_path,
    level_offsets,
    threshold_row,
    trotter_weights,
    two_field_row,
)
from . import tune  # noqa: F401,E402  (swap cadence by effective samples per second)
