"""Seeded synthetic workloads shared by the oracle and the HIP path."""
from .workloads import *  # noqa: F401,F403
