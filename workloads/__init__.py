"""Seeded synthetic LP workloads (problem data only, no solver arithmetic)."""
from .lpgen import *  # noqa: F401,F403
