"""Sequential convex programming for nonlinear covariance steering (App. F,
"Covariance Steering"), each convex step solved by the vanilla COSMO of
`solve_residual_balancing` (test infrastructure; see the package doc).

One outer iteration: linearise the dynamics at the reference (mean mu_ref,
feedforward v_ref), build the convex program with trust regions of radius
rho around the reference (synth.covsteer), solve it, and judge the step by
the ratio of the actual to the predicted decrease of the merit

    phi(z) = E-cost(z under the dynamics linearised at z) + lam_nu sum_t |d_t|_1,
    d_t = mu_{t+1} - f(mu_t, v_t)     (the nonlinear dynamics defect),

against the convex program's own value L(z) at its solution (linearised at
the reference, virtual control nu in place of d).  The step is taken when
the ratio is >= eta0; the radius halves when it is below eta1 and doubles
above eta2.  Converged when an accepted step has |d|_inf and |nu|_inf below
`tol` (the paper's 1e-3 on the nonlinear residuals).  E-cost is the
expected quadratic cost of App. F with the covariance of the disturbance
feedback K:  sum_t mu_t'Q_t mu_t + tr(Q_t Sigma_t) + v_t'R v_t +
tr(R K_t Sigma_W K_t').  The appendix prints the shrink and expand factors
(0.5, 2.0), the initial radius (5) and the tolerance; the thresholds, the
merit and the inner tolerance are readings listed with the design notes.
"""
import numpy as np

from .cosmo import solve_residual_balancing


def _transition(A_list, t, tau):
    M = np.eye(A_list[0].shape[0])
    for s in range(tau, t):
        M = A_list[s] @ M
    return M


def expected_cost(sc, A_list, B_list, mu, v, K):
    """App. F's expected cost of (mu, v, K) with the covariance propagated by
    x_{t+1} = A_t x_t + B_t u_t + w_t."""
    N = sc["N"]
    nx, nu = B_list[0].shape
    SW = np.kron(np.eye(N), sc["W"])
    f = 0.0
    for t in range(N + 1):
        Qt = sc["QN"] if t == N else sc["Q"]
        P0 = _transition(A_list, t, 0)
        Db = np.zeros((nx, N * nx))
        Bb = np.zeros((nx, N * nu))
        for tau in range(t):
            Db[:, tau * nx:(tau + 1) * nx] = _transition(A_list, t, tau + 1)
            Bb[:, tau * nu:(tau + 1) * nu] = _transition(A_list, t, tau + 1) @ B_list[tau]
        F = Db + Bb @ K
        Sig = P0 @ sc["Sigma0"] @ P0.T + F @ SW @ F.T
        f += mu[t] @ Qt @ mu[t] + np.trace(Qt @ Sig)
    for t in range(N):
        Kt = K[t * nu:(t + 1) * nu]
        f += v[t] @ sc["R"] @ v[t] + np.trace(sc["R"] @ Kt @ SW @ Kt.T)
    return float(f)


def scp(sc, step, jacobians, subproblem, unpack, mu_ref, v_ref, eps=1e-6, max_outer=30, tol=1e-3,
        eta=(0.0, 0.25, 0.75), shrink=0.5, expand=2.0, inner_max=100000):
    """Runs the outer loop from the reference (mu_ref, v_ref, K = 0).
    step(x, u), jacobians(x, u) -> (A, B): the discrete dynamics;
    subproblem(sc, mu_ref, v_ref, rho_x, rho_u) -> ConicInstance;
    unpack(inst, x) -> (mu, v, K, nu).  Returns a dict: converged, outer
    iterations, history (one record per outer iteration) and the final
    accepted (mu, v, K)."""
    N = sc["N"]
    nx = mu_ref.shape[1]
    nu = v_ref.shape[1]

    def lin(mu, v):
        AB = [jacobians(mu[t], v[t]) for t in range(N)]
        return [a for a, _ in AB], [b for _, b in AB]

    def defects(mu, v):
        return np.array([mu[t + 1] - step(mu[t], v[t]) for t in range(N)])

    K_ref = np.zeros((N * nu, N * nx))
    A_r, B_r = lin(mu_ref, v_ref)
    phi_ref = expected_cost(sc, A_r, B_r, mu_ref, v_ref, K_ref) + sc["lam_nu"] * np.abs(defects(mu_ref, v_ref)).sum()
    rho = float(sc["rho_x"])
    hist = []
    converged = False
    for it in range(max_outer):
        inst = subproblem(sc, mu_ref, v_ref, rho, rho)
        k, (x, _, _), _ = solve_residual_balancing(inst, eps_abs=eps, eps_rel=eps, max_iter=inner_max)
        mu, v, K, vn = unpack(inst, x)
        L = expected_cost(sc, A_r, B_r, mu, v, K) + sc["lam_nu"] * np.abs(vn).sum()
        A_n, B_n = lin(mu, v)
        d = defects(mu, v)
        phi_new = expected_cost(sc, A_n, B_n, mu, v, K) + sc["lam_nu"] * np.abs(d).sum()
        pred, act = phi_ref - L, phi_ref - phi_new
        ratio = act / pred if pred > 0 else float("nan")
        rec = dict(inner=k, rho=rho, phi_ref=phi_ref, phi_new=phi_new, model=L, ratio=ratio,
                   defect=float(np.abs(d).max()), nu=float(np.abs(vn).max()), accepted=False)
        hist.append(rec)
        if not pred > 1e-12 * abs(phi_ref):       # no predicted decrease left: stationary
            break
        if ratio >= eta[0]:
            rec["accepted"] = True
            mu_ref, v_ref, K_ref, A_r, B_r, phi_ref = mu, v, K, A_n, B_n, phi_new
            if rec["defect"] < tol and rec["nu"] < tol:
                converged = True
                break
        if ratio < eta[1]:
            rho *= shrink
        elif ratio > eta[2]:
            rho *= expand
    return dict(converged=converged, outer=len(hist), history=hist, mu=mu_ref, v=v_ref, K=K_ref)
