"""Seeded synthetic inputs shared by the library's tests, the bench and the oracle.

This package only draws random structure: which single-qubit gate sits where, which
couplers fire in which cycle, which bitstrings are requested and which slices are
summed.  It holds none of the method's arithmetic (no gate matrices, no contraction,
no sampling); each consumer builds its own numbers from the names and parameters
recorded here.
"""

from .circuits import (  # noqa: F401
    grid_sites,
    pattern_couplers,
    make_circuit,
    with_theta_jitter,
    circuit_from_config,
    ONEQ_NAMES,
)
from .targets import (  # noqa: F401
    bit_of,
    bitstring_from_bits,
    distinct_bitstrings,
    group_targets,
    slice_subset,
)
from .configs import CONFIGS, config  # noqa: F401
