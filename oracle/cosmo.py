"""The unrolled COSMO iteration and its reverse mode, in float64
(test infrastructure; see package doc).

An instance is any object with attributes P (n x n sparse, symmetric), q [n],
A (m x n sparse), b [m] and cones (see cones.py).

Forward step k (Sec. "Conic Operator Splitting Method", reduced form
eq:cosmo_linear_system_reduced; penalties rectified per App. E):
    rho_hat = rectify(rho^k)
    M       = P + sigma I + A' D(rho_hat) A
    xi      = sigma x - q + A'(y + rho_hat o (b - s))
    x~      = M^{-1} xi
    s~      = b - A x~            (equal to s - (y + nu~)/rho of the full system)
    x+      = alpha x~ + (1 - alpha) x
    s^      = alpha s~ + (1 - alpha) s
    s+      = Pi_K(s^ + y / rho_hat)
    y+      = y + rho_hat o (s^ - s+)
"""
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cones import proj_cone, proj_cone_vjp, rectify, rectify_adjoint


@dataclass
class Hyper:
    sigma: float = 1e-6          # fixed, Sec. "Conic Operator Splitting Method"


def reduced_matrix(inst, rho_hat: np.ndarray, sigma: float) -> sp.csc_matrix:
    """M(rho) = P + sigma I + A' D(rho) A  (eq:cosmo_linear_system_reduced)."""
    n = inst.A.shape[1]
    M = inst.P + sigma * sp.identity(n) + inst.A.T @ sp.diags(rho_hat) @ inst.A
    return sp.csc_matrix(M)


def solve_reduced(inst, rho_hat: np.ndarray, sigma: float):
    """Exact factorisation of M; returns an object with .solve(rhs)."""
    return spla.splu(reduced_matrix(inst, rho_hat, sigma))


def _keep(a):
    return a


def step_forward(inst, x, s, y, rho, alpha, sigma=1e-6, lu=None, store=_keep, solve_err=None) -> dict:
    """One COSMO step z^k -> z^{k+1}; returns every intermediate.

    store: applied to every quantity a pipeline keeps in memory as soon as it
    is formed (identity by default); solve_err(xi) -> r: the solve returns
    M^{-1}(xi + r) instead of M^{-1} xi (None: exact).  Both only serve
    unroll_forward's rounding model."""
    A, b, q = inst.A, inst.b, inst.q
    rho_hat = store(rectify(rho, inst.cones))
    if lu is None:
        lu = solve_reduced(inst, rho_hat, sigma)
    xi = sigma * x - q + A.T @ (y + rho_hat * (b - s))
    xt = store(lu.solve(xi if solve_err is None else xi + solve_err(xi)))
    st = store(b - A @ xt)
    xn = store(alpha * xt + (1.0 - alpha) * x)
    sh = store(alpha * st + (1.0 - alpha) * s)
    v = store(sh + y / rho_hat)
    sn, aux = proj_cone(v, inst.cones)
    sn = store(sn)
    if store is not _keep:
        aux = [None if a is None else (store(a[0]), store(a[1])) for a in aux]
    yn = store(y + rho_hat * (sh - sn))
    return dict(x=x, s=s, y=y, rho=rho, rho_hat=rho_hat, alpha=alpha, xi=xi, xt=xt,
                st=st, sh=sh, v=v, aux=aux, lu=lu, xn=xn, sn=sn, yn=yn)


def unroll_forward(inst, rho: np.ndarray, alpha: np.ndarray, x0=None, s0=None, y0=None,
                   sigma: float = 1e-6, store_dtype=None, store_rng=None, solve_resid: float = 0.0):
    """K steps with per-iteration (rho^k, alpha^k); z^0 = 0 unless given
    (App. D: zero default initialisation).  Returns (tape, (xK, sK, yK)).

    Rounding model (not the method; None / 0 by default).  store_dtype (e.g.
    np.float32): every per-step quantity a pipeline of that precision stores
    -- rho_hat, x~, s~, x+, s^, v, s+ with its PSD eigenpairs, y+ -- is
    rounded to it as soon as it is formed; the arithmetic stays float64.
    store_rng (a numpy Generator, with store_dtype): each stored value then
    moves by -1, 0 or +1 unit in the last place of store_dtype, uniformly at
    random -- one of the pipelines whose stored values are within one unit of
    the exact ones.  solve_resid (with store_rng): every solve stops at that
    relative residual, in a random direction.  unroll_backward runs on the
    rounded tape, so the model measures how far storage precision (and solve
    tolerance) alone move a trajectory and its gradients: a floor that a
    pipeline of that precision cannot beat."""
    n, m = inst.A.shape[1], inst.A.shape[0]
    x = np.zeros(n) if x0 is None else np.asarray(x0, np.float64).copy()
    s = np.zeros(m) if s0 is None else np.asarray(s0, np.float64).copy()
    y = np.zeros(m) if y0 is None else np.asarray(y0, np.float64).copy()
    store, solve_err = _keep, None
    if store_dtype is not None:
        dt = np.dtype(store_dtype)

        def store(a):
            r = np.asarray(a).astype(dt)
            if store_rng is not None:
                step = store_rng.integers(-1, 2, size=r.shape)
                r = np.where(step > 0, np.nextafter(r, dt.type(np.inf)),
                             np.where(step < 0, np.nextafter(r, dt.type(-np.inf)), r))
            return r.astype(np.float64)

        if store_rng is not None and solve_resid > 0:
            def solve_err(xi):
                r = store_rng.standard_normal(xi.shape)
                return r * (solve_resid * np.linalg.norm(xi) / max(np.linalg.norm(r), 1e-300))
    tape = []
    for k in range(rho.shape[0]):
        st = step_forward(inst, x, s, y, rho[k], float(alpha[k]), sigma, store=store, solve_err=solve_err)
        tape.append(st)
        x, s, y = st["xn"], st["sn"], st["yn"]
    return tape, (x, s, y)


def rounding_floor_runs(inst, rho: np.ndarray, alpha: np.ndarray, x0=None, s0=None, y0=None,
                        backward: bool = True, solve_resid: float = 0.0, store_dtype=np.float32,
                        which=(0, 1, 2)):
    """Three realisations of the rounding model (unroll_forward): stored values
    rounded to nearest with exact solves, and two (seeds 1 and 2) with every
    stored value moved by up to one unit in the last place and the solves
    stopped at solve_resid.  Returns [(x, s, y, grho, galpha)] (gradients of
    the residual loss; None when backward is False).  Against the exact run,
    the largest of their errors is the floor a pipeline storing store_dtype
    cannot beat on this instance.  which: the realisations to run."""
    out = []
    for r in which:
        kw = dict(store_dtype=store_dtype)
        if r > 0:
            kw.update(store_rng=np.random.default_rng(r), solve_resid=solve_resid)
        tape, (x, s, y) = unroll_forward(inst, rho, alpha, x0, s0, y0, **kw)
        grho = galpha = None
        if backward:
            grho, galpha, *_ = unroll_backward(inst, tape, *residual_loss_grad(inst, x, s, y))
        out.append((x, s, y, grho, galpha))
    return out


def step_backward(inst, st: dict, gxn, gsn, gyn, sigma=1e-6, gst_extra=None):
    """Reverse of one step: cotangents of (x+, s+, y+) -> cotangents of
    (x, s, y) and of (rho^k, alpha^k).  gst_extra: a cotangent of s~ from
    outside the step (the learned policy reads s~ in its delta_p feature,
    App. E), added to the step's own.

    Linear solve: with the adjoint lam~ solving M lam~ = -grad_{x~}
    (eq:grad_rho), the matrix part of the penalty gradient is
    (A lam~) o (A x~) (stacked form after eq:grad_rho).  The right-hand side
    xi also depends on (x, s, y, rho); that part (left to autograd in the
    paper) is written out by hand with xibar = M^{-1} xbar~ = -lam~.
    """
    A, b, cones = inst.A, inst.b, inst.cones
    rho_hat, alpha = st["rho_hat"], st["alpha"]
    x, s, y, xt, stl, sh, v, sn = (st[k] for k in ("x", "s", "y", "xt", "st", "sh", "v", "sn"))
    # y+ = y + rho_hat (s^ - s+)
    gy = gyn.copy()
    gsh = rho_hat * gyn
    grh = gyn * (sh - sn)
    gsn_tot = gsn - rho_hat * gyn
    # s+ = Pi_K(v)
    gv = proj_cone_vjp(v, st["aux"], cones, gsn_tot)
    # v = s^ + y / rho_hat
    gsh = gsh + gv
    gy = gy + gv / rho_hat
    grh = grh - gv * y / rho_hat ** 2
    # s^ = alpha s~ + (1 - alpha) s ;  x+ = alpha x~ + (1 - alpha) x
    gst = alpha * gsh
    if gst_extra is not None:
        gst = gst + gst_extra
    gs = (1.0 - alpha) * gsh
    galpha = float(gsh @ (stl - s) + gxn @ (xt - x))
    gx = (1.0 - alpha) * gxn
    # s~ = b - A x~
    gxt = alpha * gxn - A.T @ gst
    # x~ = M(rho)^{-1} xi
    xibar, g_mat = implicit_solve_vjp(st["lu"], A, xt, gxt)
    grh = grh + g_mat
    Axb = A @ xibar                               # xi = sigma x - q + A'(y + rho_hat (b - s))
    gx = gx + sigma * xibar
    gy = gy + Axb
    grh = grh + Axb * (b - s)
    gs = gs - rho_hat * Axb
    grho = rectify_adjoint(grh, cones)
    return gx, gs, gy, grho, galpha


def implicit_solve_vjp(lu, A, xt, gxt):
    """Matrix-free implicit differentiation of x~ = M(rho)^{-1} xi
    (Sec. "Matrix-Free Implicit Differentiation").

    The adjoint lam~ solves M lam~ = -grad_{x~} L with the same operator
    (eq:grad_rho); since dM/drho_i = a_i a_i', the penalty gradient through
    M is (A lam~) o (A x~).  The cotangent of the right-hand side is
    xibar = M^{-1} grad_{x~} L = -lam~.  Returns (xibar, grad_rho_matrix)."""
    lam = lu.solve(-gxt)                          # M symmetric
    return -lam, (A @ lam) * (A @ xt)


def unroll_backward(inst, tape: List[dict], gxK, gsK, gyK, sigma=1e-6):
    """Backpropagation through the K unrolled steps (eq:du-objective)."""
    K = len(tape)
    m = inst.A.shape[0]
    grho = np.zeros((K, m))
    galpha = np.zeros(K)
    gx, gs, gy = (np.asarray(g, np.float64).copy() for g in (gxK, gsK, gyK))
    for k in range(K - 1, -1, -1):
        gx, gs, gy, grho[k], galpha[k] = step_backward(inst, tape[k], gx, gs, gy, sigma)
    return grho, galpha, gx, gs, gy


def kkt_residuals(inst, x, s, y):
    """Primal r_p = Ax + s - b and dual r_d = Px + q - A'y.

    The paper prints the dual residual with +A'y (loss features, App. E); with the
    iteration as written the fixed point satisfies Px + q - A'y = 0
    (y lies in the polar cone), so the minus sign is the reading used."""
    rp = inst.A @ x + s - inst.b
    rd = inst.P @ x + inst.q - inst.A.T @ y
    return rp, rd


def residual_loss(inst, x, s, y) -> float:
    """Final-residual loss ||r_p||^2 + ||r_d||^2 of one instance."""
    rp, rd = kkt_residuals(inst, x, s, y)
    return float(rp @ rp + rd @ rd)


def residual_loss_grad(inst, x, s, y):
    rp, rd = kkt_residuals(inst, x, s, y)
    gx = 2.0 * (inst.A.T @ rp) + 2.0 * (inst.P.T @ rd)
    gs = 2.0 * rp
    gy = -2.0 * (inst.A @ rd)
    return gx, gs, gy


def run_fixed(inst, rho_row: np.ndarray, alpha: float, iters: int, sigma: float = 1e-6,
              z0: Optional[tuple] = None):
    """Plain COSMO with constant (rho, alpha) for `iters` steps, reusing one
    factorisation; used to reach converged values for closed-form checks."""
    n, m = inst.A.shape[1], inst.A.shape[0]
    if z0 is None:
        x, s, y = np.zeros(n), np.zeros(m), np.zeros(m)
    else:
        x, s, y = (np.asarray(z, np.float64).copy() for z in z0)
    lu = solve_reduced(inst, rectify(rho_row, inst.cones), sigma)
    for _ in range(iters):
        st = step_forward(inst, x, s, y, rho_row, alpha, sigma, lu=lu)
        x, s, y = st["xn"], st["sn"], st["yn"]
    return x, s, y


def solve_residual_balancing(inst, rho0: float = 0.1, eq_scale: float = 1e3, alpha: float = 1.6,
                             eps_abs: float = 1e-3, eps_rel: float = 1e-3, max_iter: int = 10000,
                             interval: int = 40, tol_factor: float = 5.0, rho_min: float = 1e-6,
                             rho_max: float = 1e6, adapt: bool = True, sigma: float = 1e-6, z0=None,
                             check: int = 1):
    """COSMO run to tolerance with the residual-balancing penalty: the vanilla
    baseline of Sec. "Experiments" (App. D: zero start, fixed alpha = 1.6;
    Fig. 8's caption: one scalar rho, scaled by 1e3 on equality rows).

    Stopping (checked after every step k, on z^k):
        |r_p|_inf <= eps_abs + eps_rel N_p  and  |r_d|_inf <= eps_abs + eps_rel N_d
    with r_p, r_d of kkt_residuals and the normalisers of App. E,
    N_p = max(|Ax|, |s|, |b|)_inf, N_d = max(|Px|, |q|, |A'y|)_inf.
    Penalty update (every `interval` steps, the residual-balancing rule the
    paper cites from OSQP): rho <- clip(rho sqrt((|r_p|/N_p) / (|r_d|/N_d)),
    rho_min, rho_max), taken only when it changes rho by more than a factor
    tol_factor (then M is refactorised).  The paper prints neither the rule
    nor its constants; the readings are listed with the design notes.
    check: the stopping test runs on every check-th iterate only (a solver
    that reads its residuals every few steps).  Returns (iterations, (x, s,
    y), rho) with iterations = None when max_iter steps do not reach the
    tolerance."""
    n, m = inst.A.shape[1], inst.A.shape[0]
    if z0 is None:
        x, s, y = np.zeros(n), np.zeros(m), np.zeros(m)
    else:
        x, s, y = (np.asarray(z, np.float64).copy() for z in z0)
    eq = np.zeros(m, bool)
    r = 0
    for c in inst.cones:
        rows = c.size * (c.size + 1) // 2 if c.kind == "psd" else c.size
        eq[r:r + rows] = c.kind == "zero"
        r += rows
    rho, lu = float(rho0), None
    for k in range(1, max_iter + 1):
        row = rho * np.where(eq, eq_scale, 1.0)
        if lu is None:
            lu = solve_reduced(inst, rectify(row, inst.cones), sigma)
        st = step_forward(inst, x, s, y, row, alpha, sigma, lu=lu)
        x, s, y = st["xn"], st["sn"], st["yn"]
        rp, rd = kkt_residuals(inst, x, s, y)
        Np = max(np.abs(inst.A @ x).max(initial=0.0), np.abs(s).max(initial=0.0), np.abs(inst.b).max(initial=0.0))
        Nd = max(np.abs(inst.P @ x).max(initial=0.0), np.abs(inst.q).max(initial=0.0),
                 np.abs(inst.A.T @ y).max(initial=0.0))
        ep, ed = np.abs(rp).max(initial=0.0), np.abs(rd).max(initial=0.0)
        if k % check == 0 and ep <= eps_abs + eps_rel * Np and ed <= eps_abs + eps_rel * Nd:
            return k, (x, s, y), rho
        if adapt and k % interval == 0 and Np > 0 and Nd > 0 and ed > 0:
            new = min(max(rho * np.sqrt((ep / Np) / (ed / Nd)), rho_min), rho_max)
            if new > tol_factor * rho or new < rho / tol_factor:
                rho, lu = new, None
    return None, (x, s, y), rho
