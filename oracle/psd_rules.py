"""Oracle for the alternative PSD-projection backward rules the paper compares
with the Daleckii-Krein rule (Sec. "Differentiating Through the PSD
Projection", paragraph "Alternative Approaches"; App. "Details on PSD
Projection Backward Pass Experiments").

TEST INFRASTRUCTURE ONLY (see the package docstring): float64, plain numpy,
no blocking or fusion.

  * Tikhonov: project S + eps I instead of S; the backward pass is the
    eigendecomposition rule eq:psd-cotangent applied to that matrix.
  * Newton-Schulz: Pi(S) = (S + sign(S) S) / 2 with sign(S) from the scaled
    iteration eq:newton-schulz, S_0 = S / ||S||_F, K steps; the backward pass
    is reverse mode through the K unrolled matrix products.

Reading (listed with the other readings of the paper): the number K of
Newton-Schulz steps is not printed, so it is an argument here; the output of
every rule is the symmetric part of the projected matrix, re-encoded with
svec, exactly as for eq:psd-proj, so its cotangent enters as smat(g).
"""
import numpy as np

from .cones import psd_vjp_naive
from .svec import smat, svec


def psd_vjp_tikhonov(v: np.ndarray, eps: float, gbar_svec: np.ndarray) -> np.ndarray:
    """Tikhonov rule: eigendecompose S + eps I (S = smat(v)) and apply
    eq:psd-cotangent to Pi(S + eps I) at that decomposition."""
    S = smat(v)
    lam, U = np.linalg.eigh(S + eps * np.eye(S.shape[0]))
    return psd_vjp_naive(U, lam, gbar_svec)


def ns_forward(v: np.ndarray, iters: int):
    """eq:newton-schulz on S = smat(v): S_0 = S / ||S||_F,
    S_{k+1} = 1/2 S_k (3 I - S_k^2), then Pi = (S + S_K S) / 2.
    Returns (svec of the symmetric part of Pi, tape for the reverse pass)."""
    S = smat(v)
    p = S.shape[0]
    c = float(np.linalg.norm(S, "fro"))
    X = [S / c]
    for _ in range(iters):
        Xk = X[-1]
        X.append(0.5 * Xk @ (3.0 * np.eye(p) - Xk @ Xk))
    Pi = 0.5 * (S + X[-1] @ S)
    return svec(0.5 * (Pi + Pi.T)), dict(S=S, c=c, X=X)


def ns_vjp(tape: dict, gbar_svec: np.ndarray) -> np.ndarray:
    """Reverse mode of ns_forward: the chain rule through each product of the
    unrolled iteration, last step first, then through S_0 = S / ||S||_F and
    smat.  For C = A B the cotangents are Abar = Cbar B' and Bbar = A' Cbar."""
    S, c, X = tape["S"], tape["c"], tape["X"]
    p = S.shape[0]
    I3 = 3.0 * np.eye(p)
    Tb = smat(gbar_svec)                   # cotangent of Pi (svec of sym part)
    # Pi = 1/2 S + 1/2 X_K S
    Sb = 0.5 * Tb + 0.5 * X[-1].T @ Tb
    Xb = 0.5 * Tb @ S.T
    for k in range(len(X) - 2, -1, -1):
        Xk = X[k]
        R = I3 - Xk @ Xk                   # X_{k+1} = 1/2 X_k R
        Rb = 0.5 * Xk.T @ Xb
        Xb_new = 0.5 * Xb @ R.T
        Qb = -Rb                           # R = 3 I - Q, Q = X_k X_k
        Xb_new = Xb_new + Qb @ Xk.T + Xk.T @ Qb
        Xb = Xb_new
    # X_0 = S / c with c = ||S||_F:  d(S/c) = dS / c - S <S, dS> / c^3
    Sb = Sb + Xb / c - (np.sum(Xb * S) / c ** 3) * S
    return svec(0.5 * (Sb + Sb.T))


def psd_vjp_ns(v: np.ndarray, iters: int, gbar_svec: np.ndarray) -> np.ndarray:
    """Newton-Schulz rule: forward iteration, then its reverse pass."""
    _, tape = ns_forward(v, iters)
    return ns_vjp(tape, gbar_svec)
