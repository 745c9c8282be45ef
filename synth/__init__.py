"""Seeded synthetic inputs (terrain grids) for tests and benchmarks; no viewshed arithmetic."""
from .terrain import *  # noqa: F401,F403
