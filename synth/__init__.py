"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package draws random numbers and nothing else: it holds none of the
corner-transfer arithmetic, so that neither side of a parity test can borrow
the other's contractions through it.
"""

from .tensors import (  # noqa: F401
    site_tensors,
    product_state_tensors,
    random_orthogonal,
    random_rotation2,
    serving_stream,
)
