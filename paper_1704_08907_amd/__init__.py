"""MI355X (gfx950) cell-list neighbour operators and dense kernel sums.

The hot path of the particle-based methods of Robinson & Bruna (arXiv
1704.08907): a uniform cell list (Section 2.2.1), radius-limited neighbour sums
by box search over it (Section 2.2.2, Section 3 eq. (1)), their adjoint, the
time step of the Section 3 example (eqs. (2)-(3)), and the dense kernel sum of
the RBF / Gaussian-process methods (Section 1).  The work is
done by the HIP library ``libaboria_mi355x.so``; this package binds it.
"""
from ._native import (AboriaError, BoxSpec, Cells, Context, Graph, autotune, autotune_build, autotune_cells,
                      autotune_dense,
                      build_cells, build_neighbours, cells_reorder, dense_plan_name, dense_sum, dense_sum_backward,
                      dense_sum_noalloc, graph_capture_begin, graph_capture_end, graph_launch, integrate, lib,
                      md_step, op_na, op_ny, pair_list, pair_sum, pair_sum_and_backward, pair_sum_backward,
                      selected_variant, variant_count, variant_name)

__all__ = ["AboriaError", "BoxSpec", "Cells", "Context", "Graph", "autotune", "autotune_build", "autotune_cells",
           "autotune_dense",
           "build_cells", "build_neighbours", "cells_reorder", "dense_plan_name", "dense_sum", "dense_sum_backward",
           "dense_sum_noalloc", "graph_capture_begin", "graph_capture_end", "graph_launch", "integrate", "lib",
           "md_step", "op_na", "op_ny", "pair_list", "pair_sum", "pair_sum_and_backward", "pair_sum_backward",
           "selected_variant", "variant_count", "variant_name"]
