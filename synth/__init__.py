"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the
oracle: spectral fBm terrains and observer lists.  Holds none of the siting
method's arithmetic."""
from .terrain import fbm, fbm_torch, terrain_sha256
from .observers import uniform_observers, grid_observers

__all__ = ["fbm", "fbm_torch", "terrain_sha256", "uniform_observers", "grid_observers"]
