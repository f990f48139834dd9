"""Covariance steering of a linear time-varying system as one conic program
(App. F, "Covariance Steering"): the affine disturbance-feedback
parameterisation U = K W + V, the mean dynamics with a virtual control and
its l1 epigraph, the terminal covariance bound as a Schur-complement LMI,
and optionally the trust regions of a sequential-convex-programming step.
Also the two systems of the appendix: the double integrator and the
kinematic unicycle (its dynamics, Jacobians and scenario sampler)."""
from __future__ import annotations

import math
from collections import defaultdict
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .conic import NONNEG, PSD, SOC, ZERO, Cone, ConicInstance, psd_rows, svec_index

SQRT2 = math.sqrt(2.0)


def _phi(A_list: Sequence[np.ndarray], t: int, tau: int) -> np.ndarray:
    """State-transition matrix Phi(t, tau) = A_{t-1} ... A_tau (identity when t == tau)."""
    nx = A_list[0].shape[0]
    M = np.eye(nx)
    for s in range(tau, t):
        M = A_list[s] @ M
    return M


def covsteer_ltv(A_list: Sequence[np.ndarray], B_list: Sequence[np.ndarray], r_list: Sequence[np.ndarray],
                 W: np.ndarray, mu0: np.ndarray, goal: np.ndarray, Sigma0: np.ndarray, sigma_N: float,
                 Q: np.ndarray, R: np.ndarray, QN: np.ndarray, lam_nu: float,
                 trust: Optional[Tuple[np.ndarray, np.ndarray, float, float]] = None,
                 meta: Optional[dict] = None) -> ConicInstance:
    """The convex covariance-steering program of App. F for
    x_{t+1} = A_t x_t + B_t u_t + r_t + w_t, w_t ~ N(0, W) (W diagonal),
    t = 0..N-1 (N = len(A_list)):

      min  sum_{t=0}^{N} mu_t' Q_t mu_t + tr(Q_t Sigma_t)           (Q_t = Q, Q_N = QN)
           + sum_{t<N} v_t' R v_t + tr(R K_t Sigma_W K_t') + lam_nu |nu_t|_1
      s.t. mu_{t+1} = A_t mu_t + B_t v_t + r_t + nu_t,  mu_0 = mu0,  mu_N = goal,
           Sigma_N <= sigma_N^2 I  (Schur complement, order nx + N nx),
           |mu_t - mu_ref,t| <= rho_x, |v_t - v_ref,t| <= rho_u   (trust = (mu_ref, v_ref, rho_x, rho_u))

    with Sigma_t = Phi(t,0) Sigma0 Phi(t,0)' + (Dbar_t + Bbar_t K) Sigma_W (...)', Dbar_t's
    block tau = Phi(t, tau+1), Bbar_t's block tau = Phi(t, tau+1) B_tau, K strictly
    block lower-triangular (u_t sees w_0..w_{t-1}).  Constant terms of the cost
    are dropped.  Variables: mu_0..mu_N, v_0..v_{N-1}, the blocks K[t, tau]
    (tau < t, nu x nx, row-major), nu_0..nu_{N-1}, e >= |nu| (elementwise).
    Cones: zero (mu_0, dynamics, mu_N), nonnegative (e - nu, e + nu), the trust
    regions as second-order cones (mu then v), one PSD block."""
    N = len(A_list)
    nx, nu = B_list[0].shape
    Wh = np.sqrt(np.diag(W))
    mu_off = lambda t: t * nx
    v_base = (N + 1) * nx
    v_off = lambda t: v_base + t * nu
    k_base = v_base + N * nu
    k_index: Dict[Tuple[int, int], int] = {}
    for t in range(N):
        for tau in range(t):
            k_index[(t, tau)] = k_base + len(k_index) * nu * nx
    nk = len(k_index) * nu * nx
    nu_base = k_base + nk
    e_base = nu_base + N * nx
    n = e_base + N * nx

    def kvar(t, tau, r, c):
        return k_index[(t, tau)] + r * nx + c

    phi_cache: Dict[Tuple[int, int], np.ndarray] = {}

    def phi(t, tau):
        if (t, tau) not in phi_cache:
            phi_cache[(t, tau)] = _phi(A_list, t, tau)
        return phi_cache[(t, tau)]

    def cov_factor(t):
        """(Dbar_t + Bbar_t K) Sigma_W^1/2 as a constant nx x (N nx) matrix plus
        a linear map {(row, col): {var: coef}}."""
        const = np.zeros((nx, N * nx))
        lin: Dict[Tuple[int, int], Dict[int, float]] = defaultdict(dict)
        for tau in range(t):
            const[:, tau * nx:(tau + 1) * nx] = phi(t, tau + 1) * Wh[None, :]
        for tp in range(t):                           # u_{t'} reaches x_t through Phi(t, t'+1) B_{t'}
            G = phi(t, tp + 1) @ B_list[tp]
            for tau in range(tp):
                for a in range(nx):
                    for c in range(nx):
                        for r in range(nu):
                            coef = G[a, r] * Wh[c]
                            if coef != 0.0:
                                d = lin[(a, tau * nx + c)]
                                var = kvar(tp, tau, r, c)
                                d[var] = d.get(var, 0.0) + coef
        return const, lin

    def sparse_map(lin, ncols):
        r_, c_, v_ = [], [], []
        for (a, c), terms in lin.items():
            for var, f in terms.items():
                r_.append(a * ncols + c); c_.append(var); v_.append(f)
        return sp.csr_matrix((v_, (r_, c_)), shape=(nx * ncols, n))

    Pm = sp.csr_matrix((n, n))
    qv = np.zeros(n)
    blocks_r, blocks_c, blocks_v = [], [], []
    for t in range(N + 1):
        Qt = QN if t == N else Q
        for i in range(nx):
            for j in range(nx):
                if Qt[i, j] != 0.0:
                    blocks_r.append(mu_off(t) + i); blocks_c.append(mu_off(t) + j); blocks_v.append(2.0 * Qt[i, j])
        if t >= 1:                                    # tr(Q_t Sigma_t) = |Q_t^1/2 F_t|_F^2 + const
            const, lin = cov_factor(t)
            Qh = np.linalg.cholesky(Qt).T             # Q_t = Qh' Qh
            Mq = sp.kron(sp.csr_matrix(Qh), sp.identity(N * nx), format="csr") @ sparse_map(lin, N * nx)
            cq = (Qh @ const).ravel()
            Pm = Pm + 2.0 * (Mq.T @ Mq)
            qv += 2.0 * (Mq.T @ cq)
    Rh = np.linalg.cholesky(R).T                      # R = Rh' Rh
    for t in range(N):
        for i in range(nu):
            for j in range(nu):
                if R[i, j] != 0.0:
                    blocks_r.append(v_off(t) + i); blocks_c.append(v_off(t) + j); blocks_v.append(2.0 * R[i, j])
        # tr(R K_t Sigma_W K_t') = |R^1/2 K_t Sigma_W^1/2|_F^2, K_t = block row t of K
        gr, gc, gv = [], [], []
        for tau in range(t):
            for r in range(nu):
                for c in range(nx):
                    for r2 in range(nu):
                        if Rh[r2, r] != 0.0:
                            gr.append(r2 * N * nx + tau * nx + c); gc.append(kvar(t, tau, r, c))
                            gv.append(Rh[r2, r] * Wh[c])
        if gr:
            Gm = sp.csr_matrix((gv, (gr, gc)), shape=(nu * N * nx, n))
            Pm = Pm + 2.0 * (Gm.T @ Gm)
    Pm = Pm + sp.csr_matrix((blocks_v, (blocks_r, blocks_c)), shape=(n, n))
    qv[e_base:e_base + N * nx] = lam_nu
    rows, cols, vals, b = [], [], [], []
    r = 0
    for i in range(nx):                               # mu_0 = mu0
        rows.append(r); cols.append(mu_off(0) + i); vals.append(1.0); b.append(float(mu0[i])); r += 1
    for t in range(N):                                # mu_{t+1} - A_t mu_t - B_t v_t - nu_t = r_t
        At, Bt, rt = A_list[t], B_list[t], r_list[t]
        for i in range(nx):
            rows.append(r); cols.append(mu_off(t + 1) + i); vals.append(1.0)
            for j in range(nx):
                if At[i, j] != 0.0:
                    rows.append(r); cols.append(mu_off(t) + j); vals.append(-At[i, j])
            for j in range(nu):
                if Bt[i, j] != 0.0:
                    rows.append(r); cols.append(v_off(t) + j); vals.append(-Bt[i, j])
            rows.append(r); cols.append(nu_base + t * nx + i); vals.append(-1.0)
            b.append(float(rt[i])); r += 1
    for i in range(nx):                               # mu_N = goal
        rows.append(r); cols.append(mu_off(N) + i); vals.append(1.0); b.append(float(goal[i])); r += 1
    n_zero = r
    for sgn in (-1.0, 1.0):                           # s = e + sgn nu >= 0
        for j in range(N * nx):
            rows.append(r); cols.append(e_base + j); vals.append(-1.0)
            rows.append(r); cols.append(nu_base + j); vals.append(-sgn)
            b.append(0.0); r += 1
    n_nonneg = r - n_zero
    soc_cones: List[Cone] = []
    if trust is not None:                             # s = (rho, z - z_ref) in SOC
        mu_ref, v_ref, rho_x, rho_u = trust
        for base, size, ref, rad, cnt in ((mu_off(0), nx, mu_ref, rho_x, N + 1), (v_base, nu, v_ref, rho_u, N)):
            for t in range(cnt):
                b.append(float(rad)); r += 1
                for i in range(size):
                    rows.append(r); cols.append(base + t * size + i); vals.append(-1.0)
                    b.append(-float(ref[t][i])); r += 1
                soc_cones.append(Cone(SOC, size + 1))
    # PSD: [[sigma_N^2 I - Phi(N,0) Sigma0 Phi(N,0)', F_N], [F_N', I]] >= 0
    p = nx + N * nx
    const_F, lin_F = cov_factor(N)
    PN = phi(N, 0)
    top = sigma_N ** 2 * np.eye(nx) - PN @ Sigma0 @ PN.T
    m_psd = psd_rows(p)
    bb = np.zeros(m_psd)
    prow, pcol, pval = [], [], []
    for c in range(nx):
        for a in range(c + 1):
            bb[svec_index(a, c)] += (1.0 if a == c else SQRT2) * top[a, c]
    for a in range(nx):
        for j in range(N * nx):
            idx = svec_index(a, nx + j)
            bb[idx] += SQRT2 * const_F[a, j]
            for var, coef in lin_F.get((a, j), {}).items():
                prow.append(r + idx); pcol.append(var); pval.append(-SQRT2 * coef)
    for j in range(N * nx):
        bb[svec_index(nx + j, nx + j)] += 1.0
    m = r + m_psd
    A = sp.csr_matrix((vals + pval, (rows + prow, cols + pcol)), shape=(m, n))
    A.sum_duplicates()
    bvec = np.concatenate([np.array(b), bb])
    cones = [Cone(ZERO, n_zero), Cone(NONNEG, n_nonneg)] + soc_cones + [Cone(PSD, p)]
    Pm = (0.5 * (Pm + Pm.T)).tocsr()
    Pm.sum_duplicates()
    Pm.eliminate_zeros()
    md = {"class": "covsteer_ltv", "N": N, "nx": nx, "nu": nu, "k_base": k_base, "nk": nk, "v_base": v_base,
          "nu_base": nu_base, "e_base": e_base, "Sigma_0": Sigma0, "sigma_N": sigma_N, "W": W, "goal": goal,
          "mu0": mu0, "lam_nu": lam_nu}
    if meta:
        md.update(meta)
    inst = ConicInstance(Pm, qv, A, bvec, cones, md)
    inst.check()
    return inst


def unpack_solution(inst: ConicInstance, x: np.ndarray):
    """(mu [N+1, nx], v [N, nu], K [N nu, N nx], nu [N, nx]) from the variables."""
    md = inst.meta
    N, nx, nu = md["N"], md["nx"], md["nu"]
    mu = x[:(N + 1) * nx].reshape(N + 1, nx)
    v = x[md["v_base"]:md["v_base"] + N * nu].reshape(N, nu)
    K = np.zeros((N * nu, N * nx))
    idx = md["k_base"]
    for t in range(N):
        for tau in range(t):
            K[t * nu:(t + 1) * nu, tau * nx:(tau + 1) * nx] = x[idx:idx + nu * nx].reshape(nu, nx)
            idx += nu * nx
    vn = x[md["nu_base"]:md["nu_base"] + N * nx].reshape(N, nx)
    return mu, v, K, vn


# ---- the kinematic unicycle (App. F) -------------------------------------------------

UNICYCLE_DT = 0.1
UNICYCLE_N = 30


def unicycle_step(x: np.ndarray, u: np.ndarray, dt: float = UNICYCLE_DT) -> np.ndarray:
    """Explicit Euler step of (p_x, p_y, theta)' = (v cos theta, v sin theta, omega)."""
    return x + dt * np.array([u[0] * math.cos(x[2]), u[0] * math.sin(x[2]), u[1]])


def unicycle_jacobians(x: np.ndarray, u: np.ndarray, dt: float = UNICYCLE_DT):
    """(A, B) of the Euler step at (x, u)."""
    c, s = math.cos(x[2]), math.sin(x[2])
    A = np.array([[1.0, 0.0, -dt * u[0] * s], [0.0, 1.0, dt * u[0] * c], [0.0, 0.0, 1.0]])
    B = np.array([[dt * c, 0.0], [dt * s, 0.0], [0.0, dt]])
    return A, B


def unicycle_scenario(rng: np.random.Generator, N: int = UNICYCLE_N, dt: float = UNICYCLE_DT) -> dict:
    """One scenario of App. F's unicycle class: start at the origin with
    heading ~ U[-pi, pi], target mean ~ U(-xbar, xbar) with xbar = (5, 5, pi),
    sigma_0 ~ U(0.01, 0.05), sigma_N ~ U(0.05, 0.25), W = diag(0.02^2, 0.02^2,
    0.01^2) dt, Q = diag(1, 1, 0.1), R = diag(0.1, 0.05), Q_N = 10 Q,
    lam_nu = 1e4, trust radii starting at 5."""
    mu0 = np.array([0.0, 0.0, rng.uniform(-math.pi, math.pi)])
    xbar = np.array([5.0, 5.0, math.pi])
    goal = rng.uniform(-xbar, xbar)
    s0 = rng.uniform(0.01, 0.05)
    sN = rng.uniform(0.05, 0.25)
    Q = np.diag([1.0, 1.0, 0.1])
    return dict(N=N, dt=dt, mu0=mu0, goal=goal, Sigma0=s0 ** 2 * np.eye(3), sigma_N=sN,
                W=np.diag([0.02 ** 2, 0.02 ** 2, 0.01 ** 2]) * dt, Q=Q, R=np.diag([0.1, 0.05]), QN=10.0 * Q,
                lam_nu=1e4, rho_x=5.0, rho_u=5.0)


def unicycle_subproblem(sc: dict, mu_ref: np.ndarray, v_ref: np.ndarray, rho_x: float, rho_u: float) -> ConicInstance:
    """The convex program of one SCP step: the dynamics linearised at the
    reference (mu_ref [N+1, 3], v_ref [N, 2]), r_t = f(mu_ref,t, v_ref,t) -
    A_t mu_ref,t - B_t v_ref,t, trust regions around the reference."""
    N, dt = sc["N"], sc["dt"]
    A_list, B_list, r_list = [], [], []
    for t in range(N):
        A, B = unicycle_jacobians(mu_ref[t], v_ref[t], dt)
        A_list.append(A)
        B_list.append(B)
        r_list.append(unicycle_step(mu_ref[t], v_ref[t], dt) - A @ mu_ref[t] - B @ v_ref[t])
    return covsteer_ltv(A_list, B_list, r_list, sc["W"], sc["mu0"], sc["goal"], sc["Sigma0"], sc["sigma_N"],
                        sc["Q"], sc["R"], sc["QN"], sc["lam_nu"], trust=(mu_ref, v_ref, rho_x, rho_u),
                        meta={"class": "unicycle_scp_step"})


def unicycle_initial_reference(sc: dict):
    """Straight-line reference: the mean interpolated from mu0 to the goal,
    zero controls."""
    N = sc["N"]
    lam = np.linspace(0.0, 1.0, N + 1)[:, None]
    return sc["mu0"][None, :] * (1 - lam) + sc["goal"][None, :] * lam, np.zeros((N, 2))
