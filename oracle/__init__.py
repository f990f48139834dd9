"""CPU float64 oracle for the unrolled COSMO hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call,
link or execute anything in this package: only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the HIP implementation.

It is a plain, slow, step-by-step restatement of:
  * the COSMO iteration (Sec. "Conic Operator Splitting Method",
    eq:cosmo_linear_system and the relaxation / projection / dual update that
    follow it), in the indirect (reduced) form eq:cosmo_linear_system_reduced;
  * the projections onto the zero, nonnegative, second-order and PSD cones
    (eq:psd-proj);
  * the reverse mode of K unrolled steps, with the matrix-free implicit rule
    for the linear solve (eq:grad_rho and the stacked gradient after it) and
    the Daleckii-Krein rule for the PSD projection (eq:psd-cotangent-dk,
    eq:lowner);
  * the per-block rectification of penalties (App. E, "Hyperparameter
    policy", last paragraph);
  * the final-residual training loss used by the batched max-cut workload;
  * the comparison backward rules of the PSD projection: the eigendecomposition
    rule (eq:psd-cotangent), Tikhonov-shifted and Newton-Schulz
    (eq:newton-schulz) variants;
  * the vanilla baseline: COSMO run to tolerance with the residual-balancing
    penalty (Sec. "Experiments", App. D);
  * sequential convex programming for nonlinear covariance steering (App. F),
    its convex steps solved by the vanilla baseline, in `oracle.scp`;
  * the learned hyperparameter policy inside the unroll and the log-residual
    training loss (App. E "Policy Parameterization", Sec. "Experiments"),
    in `oracle.policy`.

Precision: float64 throughout.  The linear system is solved exactly with a
sparse LU factorisation (scipy SuperLU), the tol -> 0 limit of the paper's CG.
Every function names the passage it follows; readings of silent or ambiguous
passages are listed in the design notes and repeated where used.
"""
from .svec import svec, smat, svec_len, order_from_len
from .cones import (rectify, rectify_adjoint, proj_cone, proj_cone_vjp, proj_soc, proj_soc_vjp,
                    proj_psd, psd_vjp_dk, lowner_matrix, proj_nonneg, psd_vjp_naive)
from .cosmo import (Hyper, step_forward, unroll_forward, unroll_backward, residual_loss,
                    residual_loss_grad, kkt_residuals, solve_reduced, reduced_matrix,
                    implicit_solve_vjp, step_backward, run_fixed, rounding_floor_runs,
                    solve_residual_balancing)
from .fd import fd_check_unroll, fd_directional
from .psd_rules import psd_vjp_tikhonov, ns_forward, ns_vjp, psd_vjp_ns
from . import policy, scp

__all__ = [
    "svec", "smat", "svec_len", "order_from_len",
    "rectify", "rectify_adjoint", "proj_cone", "proj_cone_vjp", "proj_soc", "proj_soc_vjp",
    "proj_psd", "psd_vjp_dk", "lowner_matrix", "proj_nonneg", "psd_vjp_naive",
    "psd_vjp_tikhonov", "ns_forward", "ns_vjp", "psd_vjp_ns",
    "Hyper", "step_forward", "unroll_forward", "unroll_backward", "residual_loss",
    "residual_loss_grad", "kkt_residuals", "solve_reduced", "reduced_matrix",
    "implicit_solve_vjp", "step_backward", "run_fixed", "rounding_floor_runs", "solve_residual_balancing",
    "fd_check_unroll", "fd_directional", "policy", "scp",
]
