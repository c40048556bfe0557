"""Exact 3D Delaunay tetrahedralization on one AMD MI355X: Python binding of libdt.so."""
from .dt import (  # noqa: F401
    DT_SCHED_LEARNED, DT_SCHED_PLAIN, DTError, Triangulation, dt_autotune, dt_clear, dt_create, dt_debug_mlp,
    dt_debug_mlp_grad, dt_debug_predicates, dt_debug_sort, dt_default_options, dt_destroy, dt_get_point_log,
    dt_get_stats, dt_get_tets, dt_get_tets_batch, dt_insert_batch, dt_insert_points, dt_load_model, dt_train_model,
    lib,
)
