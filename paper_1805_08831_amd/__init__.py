"""Exact 3D Delaunay tetrahedralization on one AMD MI355X: Python binding of libdt.so."""
from .dt import (  # noqa: F401
    DTError, Triangulation, dt_clear, dt_create, dt_debug_predicates, dt_debug_sort,
    dt_default_options, dt_destroy, dt_get_stats, dt_get_tets, dt_insert_points, lib,
)
