"""Cone projections, their vector-Jacobian products, and penalty
rectification (test infrastructure; see package doc).

Cones are given as a list of objects with `.kind` in {"zero", "nonneg",
"soc", "psd"} and `.size` (rows, or the matrix order p for "psd"); rows of
the stacked vector follow the list order.
"""
import math

import numpy as np

from .svec import smat, svec, svec_len


def _rows(c) -> int:
    return svec_len(c.size) if c.kind == "psd" else c.size


def _blocks(cones):
    r = 0
    for c in cones:
        d = _rows(c)
        yield c, slice(r, r + d)
        r += d


# --- rectification (App. E "Hyperparameter policy", final paragraph) -------

def rectify(rho: np.ndarray, cones) -> np.ndarray:
    """Average the per-row penalties inside every SOC and PSD block and
    broadcast the mean back; zero and nonnegative rows keep their own."""
    out = np.array(rho, dtype=np.float64, copy=True)
    for c, sl in _blocks(cones):
        if c.kind in ("soc", "psd"):
            out[sl] = np.mean(rho[sl])
    return out


def rectify_adjoint(g_hat: np.ndarray, cones) -> np.ndarray:
    """Adjoint of `rectify`: d rho_hat_r / d rho_j = 1/d inside a block, so
    every row of the block receives the block mean of the incoming cotangent."""
    out = np.array(g_hat, dtype=np.float64, copy=True)
    for c, sl in _blocks(cones):
        if c.kind in ("soc", "psd"):
            out[sl] = np.mean(g_hat[sl])
    return out


# --- projections (eq:cosmo_projection, eq:psd-proj) -------------------------

def proj_nonneg(v):
    return np.maximum(v, 0.0)


def proj_soc(v: np.ndarray) -> np.ndarray:
    """Euclidean projection onto {(t, w): ||w|| <= t} (textbook closed form;
    the paper calls these projections smooth or piecewise smooth, Sec.
    "Stable PSD Projection").  Boundary ties take the identity/zero branch."""
    t, w = v[0], v[1:]
    nw = float(np.linalg.norm(w))
    if nw <= t:
        return v.copy()
    if nw <= -t:
        return np.zeros_like(v)
    a = 0.5 * (1.0 + t / nw)
    return np.concatenate([[a * nw], a * w])


def proj_psd(v: np.ndarray):
    """eq:psd-proj on an svec block: eigendecompose smat(v), clip negative
    eigenvalues, rebuild, re-encode.  Returns (svec(Pi), U, lam)."""
    S = smat(v)
    lam, U = np.linalg.eigh(S)
    T = (U * np.maximum(lam, 0.0)) @ U.T
    return svec(0.5 * (T + T.T)), U, lam


def proj_cone(v: np.ndarray, cones):
    """Pi_K for the product cone; also returns per-block data the reverse
    mode needs (eigendecompositions of PSD blocks)."""
    out = np.empty_like(v)
    aux = []
    for c, sl in _blocks(cones):
        if c.kind == "zero":
            out[sl] = 0.0
            aux.append(None)
        elif c.kind == "nonneg":
            out[sl] = proj_nonneg(v[sl])
            aux.append(None)
        elif c.kind == "soc":
            out[sl] = proj_soc(v[sl])
            aux.append(None)
        elif c.kind == "psd":
            out[sl], U, lam = proj_psd(v[sl])
            aux.append((U, lam))
        else:
            raise ValueError(c.kind)
    return out, aux


# --- vector-Jacobian products ----------------------------------------------

def proj_soc_vjp(v: np.ndarray, g: np.ndarray) -> np.ndarray:
    """J(v)' g for the SOC projection.  Interior of the cone: J = I; interior
    of the polar cone: J = 0; otherwise, with nu = ||w||, u = w / nu,
    J = 1/2 [[1, u'], [u, (1 + t/nu) I - (t/nu) u u']] (symmetric)."""
    t, w = v[0], v[1:]
    nw = float(np.linalg.norm(w))
    if nw <= t:
        return g.copy()
    if nw <= -t:
        return np.zeros_like(g)
    u = w / nw
    d = len(v)
    J = np.zeros((d, d))
    J[0, 0] = 1.0
    J[0, 1:] = u
    J[1:, 0] = u
    J[1:, 1:] = (1.0 + t / nw) * np.eye(d - 1) - (t / nw) * np.outer(u, u)
    return 0.5 * (J.T @ g)


def lowner_matrix(lam: np.ndarray) -> np.ndarray:
    """eq:lowner for f(x) = max(x, 0): first divided differences of f at the
    eigenvalues, f'(lam_i) on ties, with f'(0) taken as 0."""
    f = np.maximum(lam, 0.0)
    p = len(lam)
    L = np.empty((p, p))
    for i in range(p):
        for j in range(p):
            if lam[i] != lam[j]:
                L[i, j] = (f[j] - f[i]) / (lam[j] - lam[i])
            else:
                L[i, j] = 1.0 if lam[i] > 0.0 else 0.0
    return L


def psd_vjp_dk(U: np.ndarray, lam: np.ndarray, gbar_svec: np.ndarray) -> np.ndarray:
    """eq:psd-cotangent-dk in svec coordinates: Sbar = U (L o (U' Tbar U)) U'
    with Tbar = smat(gbar); svec's adjoint is smat, so the input cotangent is
    svec(Sbar)."""
    Tb = smat(gbar_svec)
    Sb = U @ (lowner_matrix(lam) * (U.T @ Tb @ U)) @ U.T
    return svec(0.5 * (Sb + Sb.T))


def psd_vjp_naive(U: np.ndarray, lam: np.ndarray, gbar_svec: np.ndarray) -> np.ndarray:
    """eq:psd-cotangent: the eigendecomposition rule autograd applies to
    T = U max(L, 0) U'.  Kept as the unstable comparison: F_ij = 1/(l_j - l_i)
    is infinite on repeated eigenvalues."""
    Tb = smat(gbar_svec)
    f = np.maximum(lam, 0.0)
    df = (lam > 0).astype(np.float64)
    Ubar = 2.0 * Tb @ U * f                       # d<Tb, U f U'>/dU
    lbar = np.diag(U.T @ Tb @ U) * df             # d/dlam
    diff = lam[None, :] - lam[:, None]            # lam_j - lam_i
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(np.eye(len(lam), dtype=bool), 0.0, 1.0 / diff)
    inner = np.diag(lbar) + F * (U.T @ Ubar)
    Sb = U @ inner @ U.T
    return svec(0.5 * (Sb + Sb.T))


def proj_cone_vjp(v: np.ndarray, aux, cones, g: np.ndarray) -> np.ndarray:
    """J_Pi(v)' g block by block (zero: 0; nonneg: mask v > 0, so the kink
    at 0 takes derivative 0; SOC; PSD by Daleckii-Krein)."""
    out = np.empty_like(g)
    for (c, sl), a in zip(_blocks(cones), aux):
        if c.kind == "zero":
            out[sl] = 0.0
        elif c.kind == "nonneg":
            out[sl] = g[sl] * (v[sl] > 0.0)
        elif c.kind == "soc":
            out[sl] = proj_soc_vjp(v[sl], g[sl])
        else:
            U, lam = a
            out[sl] = psd_vjp_dk(U, lam, g[sl])
    return out


def active_signature(v: np.ndarray, cones):
    """Which smooth piece of Pi_K holds at v: nonneg signs, SOC case, PSD
    inertia.  Used by the finite-difference driver to skip kinks."""
    sig = []
    for c, sl in _blocks(cones):
        if c.kind == "nonneg":
            sig.append(tuple((v[sl] > 0).tolist()))
        elif c.kind == "soc":
            t, w = v[sl][0], v[sl][1:]
            nw = float(np.linalg.norm(w))
            sig.append(0 if nw <= t else (1 if nw <= -t else 2))
        elif c.kind == "psd":
            lam = np.linalg.eigvalsh(smat(v[sl]))
            sig.append(int(np.sum(lam > 0)))
    return tuple(sig)
