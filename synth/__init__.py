"""Seeded synthetic inputs (objects, projections, intensities, supports).

Serves both the CPU oracle and the GPU path; holds none of the
reconstruction method's arithmetic.
"""
from .configs import make_scan, angles, build_object  # noqa: F401
