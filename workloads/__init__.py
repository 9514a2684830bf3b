"""Seeded synthetic inputs shared by the oracle and the GPU path (no method arithmetic)."""
from . import surfaces, configs  # noqa: F401
