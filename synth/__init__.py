"""Seeded synthetic conic-program generators.

This package builds problem data only: instances d = (P, q, A, b, K) of the
standard conic form of Sec. "Deep Unfolding Conic Optimization"
(eq:conic-standard), plus the seeded hyperparameter sequences (rho^k, alpha^k)
fed to the unrolled solver.  It holds none of the solver's arithmetic (no
linear solve, no projection, no gradient) and is shared by the CPU oracle's
tests and by the GPU path's tests and benchmark.
"""
from .conic import ConicInstance, Cone, psd_rows, svec_index, svec_of_dense, cone_row_slices
from .graphs import erdos_renyi, circulant, complete_graph, cycle_graph, petersen_graph
from .problems import maxcut_sdp, lovasz_theta_sdp, huber_socp, covsteer_sdp, double_integrator_cs, random_mixed
from .workloads import (c1_instance, c2_batch, c3_batch, c4_batch, c5_batch,
                        default_rho, perturbed_hyper, appb_instance, appc_matrix)

__all__ = [
    "ConicInstance", "Cone", "psd_rows", "svec_index", "svec_of_dense", "cone_row_slices",
    "erdos_renyi", "circulant", "complete_graph", "cycle_graph", "petersen_graph",
    "maxcut_sdp", "lovasz_theta_sdp", "huber_socp", "covsteer_sdp", "double_integrator_cs", "random_mixed",
    "c1_instance", "c2_batch", "c3_batch", "c4_batch", "c5_batch",
    "default_rho", "perturbed_hyper", "appb_instance", "appc_matrix",
]
