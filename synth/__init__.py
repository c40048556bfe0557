"""Seeded synthetic point clouds shared by the tests, the benchmark and the oracle runs.

This module only draws random inputs; it holds none of the triangulation's arithmetic.
"""
from .generators import (  # noqa: F401
    splitmix64,
    uniform_points,
    lattice_points,
    cluster_points,
    shell_points,
    mix_points,
    batch_clouds,
)
