"""Conic encodings of the problem classes of App. F (and the readings used
for the Huber-regression SOCP and the covariance-steering SDP).

Every builder returns a ConicInstance in the standard form of
eq:conic-standard.  Maximisations are written as minimisations of the
negated objective, so a converged objective q'x equals minus the SDP value.
"""
from __future__ import annotations

import math
from collections import defaultdict
from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .conic import NONNEG, PSD, SOC, ZERO, Cone, ConicInstance, psd_rows, svec_index

SQRT2 = math.sqrt(2.0)


def _svec_of_dense(X: np.ndarray) -> np.ndarray:
    p = X.shape[0]
    out = np.empty(psd_rows(p))
    for j in range(p):
        for i in range(j + 1):
            out[svec_index(i, j)] = X[i, j] if i == j else SQRT2 * X[i, j]
    return out


def _laplacian(n: int, edges, weights=None) -> np.ndarray:
    L = np.zeros((n, n))
    for e, (i, j) in enumerate(edges):
        w = 1.0 if weights is None else weights[e]
        L[i, j] -= w
        L[j, i] -= w
        L[i, i] += w
        L[j, j] += w
    return L


def maxcut_sdp(n: int, edges, weights=None) -> ConicInstance:
    """App. F max-cut: maximise 1/4 <L, X> s.t. X_ii = 1, X psd.

    Variables x = svec(X).  Rows: n zero-cone rows selecting svec(X)_(i,i)
    (b = 1), then p(p+1)/2 PSD rows with A = -I, b = 0, so s = svec(X).
    """
    nv = psd_rows(n)
    L = _laplacian(n, edges, weights)
    q = -0.25 * _svec_of_dense(L)
    rows, cols, vals = [], [], []
    for i in range(n):
        rows.append(i); cols.append(svec_index(i, i)); vals.append(1.0)
    for k in range(nv):
        rows.append(n + k); cols.append(k); vals.append(-1.0)
    m = n + nv
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, nv))
    b = np.zeros(m); b[:n] = 1.0
    P = sp.csr_matrix((nv, nv))
    inst = ConicInstance(P, q, A, b, [Cone(ZERO, n), Cone(PSD, n)],
                         {"class": "maxcut", "order": n, "edges": list(edges)})
    inst.check()
    return inst


def lovasz_theta_sdp(n: int, edges) -> ConicInstance:
    """App. F Lovasz theta: maximise <J, X> s.t. tr X = 1, X_ij = 0 on edges,
    X psd.  Rows: 1 + |E| zero-cone rows, then the PSD block (A = -I)."""
    nv = psd_rows(n)
    q = -_svec_of_dense(np.ones((n, n)))
    rows, cols, vals = [], [], []
    for i in range(n):                       # tr X = <I, X> = svec(I)' x
        rows.append(0); cols.append(svec_index(i, i)); vals.append(1.0)
    for e, (i, j) in enumerate(edges):       # svec entry of X_ij is sqrt2 X_ij
        rows.append(1 + e); cols.append(svec_index(i, j)); vals.append(1.0)
    nz = 1 + len(edges)
    for k in range(nv):
        rows.append(nz + k); cols.append(k); vals.append(-1.0)
    m = nz + nv
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, nv))
    b = np.zeros(m); b[0] = 1.0
    P = sp.csr_matrix((nv, nv))
    inst = ConicInstance(P, q, A, b, [Cone(ZERO, nz), Cone(PSD, n)],
                         {"class": "lovasz", "order": n, "edges": list(edges)})
    inst.check()
    return inst


def huber_socp(rng: np.random.Generator, n_obs: int = 2000, n_coef: int = 500,
               n_soc: int = 200, soc_dims=(3, 10), delta: float = 1.345) -> ConicInstance:
    """Huber regression with Student-t(2) noise plus group-norm SOC limits.

    Huber (App. F robust Kalman class): phi_d(r) = min_u u^2 + 2d|r - u|.
    z = (beta, u, w); P = diag(0, 2I, 0); q = (0, 0, 2d 1).
    Nonneg rows:  [ G, -I, -I] z + s = b    and   [-G,  I, -I] z + s = -b,
    i.e. |G beta - b - u| <= w.  SOC j: ||beta_{S_j}|| <= c_j with S_j a random
    (d_j - 1)-subset of the coefficients and c_j = U(0.5, 1.5) ||beta_true,S_j||.
    """
    G = rng.standard_normal((n_obs, n_coef))
    beta = rng.standard_normal(n_coef)
    bobs = G @ beta + rng.standard_t(2.0, size=n_obs)
    n = n_coef + 2 * n_obs
    I = sp.identity(n_obs, format="csr")
    Gs = sp.csr_matrix(G)
    top = sp.hstack([Gs, -I, -I])
    mid = sp.hstack([-Gs, I, -I])
    dims = rng.integers(soc_dims[0], soc_dims[1] + 1, size=n_soc)
    srows, scols, svals, sb = [], [], [], []
    r = 0
    for d in dims:
        S = rng.choice(n_coef, size=d - 1, replace=False)
        c = rng.uniform(0.5, 1.5) * float(np.linalg.norm(beta[S]))
        sb.append(c)
        for t, g in enumerate(S):
            srows.append(r + 1 + t); scols.append(int(g)); svals.append(-1.0)
            sb.append(0.0)
        r += int(d)
    socA = sp.csr_matrix((svals, (srows, scols)), shape=(r, n))
    A = sp.vstack([top, mid, socA]).tocsr()
    b = np.concatenate([bobs, -bobs, np.array(sb)])
    pdiag = np.concatenate([np.zeros(n_coef), 2.0 * np.ones(n_obs), np.zeros(n_obs)])
    P = sp.diags(pdiag).tocsr()
    q = np.concatenate([np.zeros(n_coef + n_obs), 2.0 * delta * np.ones(n_obs)])
    cones = [Cone(NONNEG, 2 * n_obs)] + [Cone(SOC, int(d)) for d in dims]
    inst = ConicInstance(P, q, A, b, cones,
                         {"class": "huber", "n_obs": n_obs, "n_coef": n_coef,
                          # the design G sits at rows 0.. and (negated) at rows n_obs..
                          "dense": {"col0": 0, "rows": n_obs, "cols": n_coef,
                                    "place": [(0, 1.0), (n_obs, -1.0)]}})
    inst.check()
    return inst


class _LmiBuilder:
    """Accumulates affine PSD constraints  Lin(x) + C  >= 0  into rows
    A x + s = b with s = svec(Lin(x) + C):  A = -svec(Lin), b = svec(C)."""

    def __init__(self) -> None:
        self.rows: List[int] = []
        self.cols: List[int] = []
        self.vals: List[float] = []
        self.b: List[float] = []
        self.cones: List[Cone] = []
        self.m = 0

    def add_block(self, p: int, lin: Dict[Tuple[int, int], Dict[int, float]],
                  const: Dict[Tuple[int, int], float]) -> None:
        base = self.m
        nr = psd_rows(p)
        bb = np.zeros(nr)
        for (i, j), c in const.items():
            sc = 1.0 if i == j else SQRT2
            bb[svec_index(i, j)] += sc * c
        for (i, j), terms in lin.items():
            sc = 1.0 if i == j else SQRT2
            r = base + svec_index(i, j)
            for var, coef in terms.items():
                if coef != 0.0:
                    self.rows.append(r); self.cols.append(var); self.vals.append(-sc * coef)
        self.b.extend(bb.tolist())
        self.cones.append(Cone(PSD, p))
        self.m += nr


def covsteer_sdp(rng: np.random.Generator, nx: int, T: int, w_scale: float = 0.01) -> ConicInstance:
    """Linear covariance-steering SDP with per-step LMI blocks (App. F CS
    class, Schur-complement form).  nu = nx/2.

    Variables: Sigma_1..Sigma_T (svec, order nx), U_0..U_{T-1} (nu x nx,
    row-major), Y_0..Y_{T-1} (svec, order nu).  Sigma_0 is data.
    Blocks for k = 0..T-1:
      [[Sigma_k, U_k'], [U_k, Y_k]] >= 0                      (order nx+nu)
      [[Sigma_{k+1} - W, A_k Sigma_k + B_k U_k], [., Sigma_k]] >= 0  (order 2nx)
    and the terminal block Sigma_term - Sigma_T >= 0 (order nx).
    Objective sum_k tr(Sigma_k) + tr(Y_k) (Q = R = I).
    """
    nu = nx // 2
    ns, ny = psd_rows(nx), psd_rows(nu)
    sig_off = {k: (k - 1) * ns for k in range(1, T + 1)}
    u_base = T * ns
    u_off = {k: u_base + k * nu * nx for k in range(T)}
    y_base = u_base + T * nu * nx
    y_off = {k: y_base + k * ny for k in range(T)}
    n = y_base + T * ny

    def wishart():
        Gw = rng.standard_normal((nx, nx + 2))
        return Gw @ Gw.T / (nx + 2)

    Sig0, Sterm = wishart(), wishart()
    Ak, Bk = [], []
    for _ in range(T):
        Gm = rng.standard_normal((nx, nx))
        rad = max(abs(np.linalg.eigvals(Gm)))
        Ak.append(rng.uniform(0.95, 1.05) * Gm / rad)
        Bk.append(rng.standard_normal((nx, nu)))
    W = w_scale * np.eye(nx)

    def sig_term(k, a, c):
        """(linear terms, constant) of Sigma_k[a, c]."""
        if k == 0:
            return {}, Sig0[a, c]
        f = 1.0 if a == c else 1.0 / SQRT2
        return {sig_off[k] + svec_index(a, c): f}, 0.0

    bld = _LmiBuilder()
    for k in range(T):
        # block 1: [[Sigma_k, U_k'], [U_k, Y_k]]
        p = nx + nu
        lin, const = defaultdict(dict), defaultdict(float)
        for c in range(nx):
            for a in range(c + 1):
                t, cst = sig_term(k, a, c)
                lin[(a, c)].update(t); const[(a, c)] += cst
        for r in range(nu):
            for c in range(nx):
                lin[(c, nx + r)][u_off[k] + r * nx + c] = 1.0
        for t2 in range(nu):
            for r in range(t2 + 1):
                f = 1.0 if r == t2 else 1.0 / SQRT2
                lin[(nx + r, nx + t2)][y_off[k] + svec_index(r, t2)] = f
        bld.add_block(p, lin, const)
        # block 2: [[Sigma_{k+1} - W, A Sigma_k + B U_k], [., Sigma_k]]
        p = 2 * nx
        lin, const = defaultdict(dict), defaultdict(float)
        for c in range(nx):
            for a in range(c + 1):
                t, cst = sig_term(k + 1, a, c)
                lin[(a, c)].update(t); const[(a, c)] += cst - W[a, c]
                t, cst = sig_term(k, a, c)
                lin[(nx + a, nx + c)].update(t); const[(nx + a, nx + c)] += cst
        A_, B_ = Ak[k], Bk[k]
        for a in range(nx):
            for c in range(nx):
                ent = lin[(a, nx + c)]
                for l in range(nx):
                    t, cst = sig_term(k, l, c)
                    for var, f in t.items():
                        ent[var] = ent.get(var, 0.0) + A_[a, l] * f
                    const[(a, nx + c)] += A_[a, l] * cst
                for r in range(nu):
                    var = u_off[k] + r * nx + c
                    ent[var] = ent.get(var, 0.0) + B_[a, r]
        bld.add_block(p, lin, const)
    # terminal: Sigma_term - Sigma_T
    lin, const = defaultdict(dict), defaultdict(float)
    for c in range(nx):
        for a in range(c + 1):
            t, _ = sig_term(T, a, c)
            lin[(a, c)].update({v: -f for v, f in t.items()})
            const[(a, c)] += Sterm[a, c]
    bld.add_block(nx, lin, const)

    A = sp.csr_matrix((bld.vals, (bld.rows, bld.cols)), shape=(bld.m, n))
    A.sum_duplicates()
    b = np.array(bld.b)
    q = np.zeros(n)
    for k in range(1, T + 1):
        for a in range(nx):
            q[sig_off[k] + svec_index(a, a)] = 1.0
    for k in range(T):
        for r in range(nu):
            q[y_off[k] + svec_index(r, r)] = 1.0
    P = sp.csr_matrix((n, n))
    inst = ConicInstance(P, q, A, b, bld.cones, {"class": "covsteer", "nx": nx, "nu": nu, "T": T})
    inst.check()
    return inst


def double_integrator_cs(rng: np.random.Generator, N: int = 10, dt: float = 0.5, sigma_a: float = 0.3,
                         sigma_0: float = 0.01, sigma_N: float = 0.25, lam_nu: float = 100.0,
                         goal_box=(5.0, 5.0)) -> ConicInstance:
    """Covariance steering of the 2D double integrator (App. F, "Covariance
    Steering"), the convex program of the affine disturbance-feedback
    parameterisation U = K W + V: state (p_x, p_y, v_x, v_y), control
    (a_x, a_y), exact zero-order-hold A, B and the noise covariance W of the
    appendix; mean mu_0 = 0, target mean (position ~ U(-goal_box, goal_box),
    velocity 0); Sigma_0 = sigma_0^2 I, terminal bound Sigma_N <= sigma_N^2 I
    (the isotropic constraint whose active eigenvalues coalesce); costs
    Q = diag(1, 1, 0.3, 0.3), R = 0.1 I, Q_N = 10 Q on means and covariances;
    a virtual control nu_t on the mean dynamics with an l1 penalty lam_nu.
    The appendix gives neither the step dt, the noise scale sigma_a, lam_nu
    nor an intermediate bound Sigma_max; only the terminal LMI is imposed.
    The last step's noise cannot be fed back (u_t sees w_0..w_{t-1}), so the
    bound is feasible only while dt sigma_a^2 < sigma_N^2 (sigma_a < 0.354 at
    dt = 0.5); the default 0.3 is feasible, and its solution is strictly
    inside the bound.

    Variables: mu_0..mu_N, v_0..v_{N-1}, the strictly block lower-triangular
    K (blocks K[t, tau], tau < t, nu x nx, row-major), nu_t, and epigraph
    variables e >= |nu|.  Rows: zero cone (mu_0 = 0, mean dynamics,
    mu_N = goal), nonnegative cone (e - nu, e + nu), and one PSD block of
    order nx + N nx: the Schur complement of
    sigma_N^2 I - A^N Sigma_0 A^N' - (Dbar_N + Bbar_N K) Sigma_W (...)' >= 0."""
    from .covsteer import covsteer_ltv
    nx, nu = 4, 2
    I2 = np.eye(2)
    A = np.block([[I2, dt * I2], [np.zeros((2, 2)), I2]])
    B = np.vstack([0.5 * dt * dt * I2, dt * I2])
    W = np.diag([dt ** 3 / 3 * sigma_a ** 2] * 2 + [dt * sigma_a ** 2] * 2)
    Sig0 = sigma_0 ** 2 * np.eye(nx)
    Q = np.diag([1.0, 1.0, 0.3, 0.3])
    goal = np.concatenate([rng.uniform(-np.asarray(goal_box), np.asarray(goal_box)), np.zeros(2)])
    return covsteer_ltv([A] * N, [B] * N, [np.zeros(nx)] * N, W, np.zeros(nx), goal, Sig0, sigma_N, Q,
                        0.1 * np.eye(nu), 10.0 * Q, lam_nu,
                        meta={"class": "double_integrator_cs", "dt": dt, "sigma_a": sigma_a, "A": A, "B": B})


def random_mixed(rng: np.random.Generator, n: int = 8, n_zero: int = 2, n_nonneg: int = 3,
                 soc_dims=(3,), psd_orders=(3,), density: float = 0.6) -> ConicInstance:
    """Small random instance mixing all four cone types (for derivative and
    parity checks).  P = G G' / n is positive semidefinite; A has random
    sparsity with every row non-empty; b and q are Gaussian."""
    cones = []
    if n_zero:
        cones.append(Cone(ZERO, n_zero))
    if n_nonneg:
        cones.append(Cone(NONNEG, n_nonneg))
    cones += [Cone(SOC, d) for d in soc_dims] + [Cone(PSD, p) for p in psd_orders]
    m = sum(c.rows for c in cones)
    Gp = rng.standard_normal((n, n // 2 + 1))
    Pd = Gp @ Gp.T / n
    mask = rng.random((m, n)) < density
    mask[np.arange(m), rng.integers(0, n, size=m)] = True
    Ad = np.where(mask, rng.standard_normal((m, n)), 0.0)
    inst = ConicInstance(sp.csr_matrix(Pd), rng.standard_normal(n), sp.csr_matrix(Ad),
                         rng.standard_normal(m), cones, {"class": "mixed"})
    inst.check()
    return inst
