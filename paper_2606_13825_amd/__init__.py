"""MI355X-native batched, unrolled COSMO for conic programs.

Forward: matrix-free Jacobi-PCG on the reduced system, projections onto the
zero, nonnegative, second-order and PSD cones.  Backward: adjoint PCG
(matrix-free implicit differentiation) and the Daleckii-Krein VJP of the PSD
projection; the paper's comparison backward rules of the PSD projection
(eigendecomposition rule, Tikhonov shift, Newton-Schulz); the learned
hyperparameter policy inside the unroll with the log-residual loss; the
vanilla COSMO run to tolerance.  All of it runs in the HIP library
libcosmo_unroll.so behind the C ABI of include/cosmo_unroll.h; this package
only marshals arguments.  `scp` drives sequential convex programming for
nonlinear covariance steering around batched vanilla solves (its outer
ratio test runs on the host).
"""
from .binding import (CosmoBatch, CosmoUnroll, ResidualLoss, psd_proj, psd_proj_vjp, socp_proj,
                      socp_proj_vjp, ForwardResult, BackwardResult, psd_proj_vjp_rule, NewtonSchulzProj,
                      PolicyForwardResult, policy_init)
from ._lib import CosmoError, lib, LIB_PATH
from . import scp
from .scp import scp_solve, ScpResult, ScpTiming

__all__ = ["CosmoBatch", "CosmoUnroll", "ResidualLoss", "psd_proj", "psd_proj_vjp", "socp_proj",
           "socp_proj_vjp", "ForwardResult", "BackwardResult", "CosmoError", "lib", "LIB_PATH",
           "psd_proj_vjp_rule", "NewtonSchulzProj", "PolicyForwardResult", "policy_init",
           "scp", "scp_solve", "ScpResult", "ScpTiming"]
