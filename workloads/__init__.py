"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no part of the method's arithmetic: it only draws random
numbers and arranges them into integral tensors and flat value streams.  Both
the CPU oracle and the HIP library consume exactly these arrays.
"""

from .integrals import (  # noqa: F401
    Integrals,
    random_molecule_integrals,
    chain_integrals,
    workload_integrals,
    batched_instances,
    mps_values,
    separable_integrals,
    nearest_neighbour_integrals,
    exponential_density_integrals,
    WORKLOADS,
)
