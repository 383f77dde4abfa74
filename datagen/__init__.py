"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws inputs.  It holds none of the method's arithmetic
(no hashing, no pair enumeration, no counting); both the CPU oracle and the
GPU library consume what it returns.
"""
from .streams import (  # noqa: F401
    Raw,
    Transactions,
    OuterProducts,
    transactions,
    outer_products,
    config_small,
    config_large,
    config_outer,
    config_batched,
    config_batched_stream,
    config_learned_train,
    config_learned_heldout,
    tiny_transactions,
    tiny_outer,
    concat_transactions,
    mlp_init_weights,
    sample_order,
)
