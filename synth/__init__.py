"""Seeded synthetic inputs shared by the oracle and the GPU library."""
from . import mesh, scenarios  # noqa: F401
