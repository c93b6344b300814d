"""Seeded synthetic workloads (circuit descriptions) used by the tests and the benchmark."""
from .circuit import Circuit, Op  # noqa: F401
