"""Seeded synthetic inputs (systems and model parameters) for the REANN path.

This package is the only code that the oracle tests and the GPU path share: it
draws inputs and holds none of the model's arithmetic.
"""
from . import models, systems  # noqa: F401
from .workloads import WORKLOADS, workload  # noqa: F401
