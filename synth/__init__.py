"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the bench.

Holds none of the method's arithmetic: only media (slowness kappa), sources and the
frequency implied by a points-per-wavelength target.
"""
from .media import (  # noqa: F401
    homogeneous, layered_2d, geophysical_3d, linear_kappa2, point_source,
    omega_for_ppw, random_sources,
)
