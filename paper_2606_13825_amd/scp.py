"""Sequential convex programming for nonlinear covariance steering (App. F,
"Covariance Steering") with every convex step solved on the GPU by the
vanilla COSMO of `CosmoBatch.solve` (residual-balancing penalty).

The scenarios of a call advance in lock step: each outer iteration gathers
the convex programs of the scenarios still running into one super-batch,
solves it in one `cosmo_solve`, and then runs each scenario's trust-region
ratio test on the host.  The problem definition comes in as callables, so
this module knows nothing of a particular system:

  step(x, u) -> x_next               the discrete dynamics f,
  jacobians(x, u) -> (A, B)          its Jacobians,
  subproblem(sc, mu_ref, v_ref, rho_x, rho_u) -> conic instance
                                     the convex program linearised at the
                                     reference, with trust regions,
  unpack(inst, x) -> (mu, v, K, nu)  mean, feedforward, disturbance feedback
                                     and virtual control from its solution,
  reference(sc) -> (mu_ref, v_ref)   the initial reference.

A scenario `sc` is a dict with N, Sigma0, W, Q, R, QN, lam_nu and the initial
trust radius rho_x.  The step is judged by the ratio of the actual decrease
of the merit

    phi(z) = E-cost of z (covariance propagated by the dynamics linearised at z)
             + lam_nu sum_t |mu_{t+1} - f(mu_t, v_t)|_1

to the decrease the convex program predicts (its objective at the solution,
linearised at the reference, with the virtual control in place of the
defect).  Ratio >= eta[0] accepts; below eta[1] the radius shrinks, above
eta[2] it expands.  A scenario has converged when an accepted step leaves
the nonlinear defect and the virtual control below `tol` in max-norm.  The
appendix gives the shrink and expand factors, the initial radius and the
tolerance; the merit, the thresholds and the inner tolerance are readings.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Sequence

import numpy as np
import torch

from .binding import CosmoBatch


def expected_cost(sc: dict, A_list, B_list, mu: np.ndarray, v: np.ndarray, K: np.ndarray) -> float:
    """The expected quadratic cost of App. F for the affine disturbance
    feedback u_t = v_t + sum_{tau<t} K_{t,tau} w_tau under
    x_{t+1} = A_t x_t + B_t u_t + w_t:

      sum_{t<=N} mu_t'Q_t mu_t + tr(Q_t Sigma_t) + sum_{t<N} v_t'R v_t + tr(R K_t S_W K_t')

    (Q_N for the last state).  Sigma_t is carried forward: the state's
    deviation is Phi_t dx_0 + F_t w with F_{t+1} = A_t F_t + B_t K_t + E_t
    (E_t picks w_t), so Sigma_t = Phi_t Sigma_0 Phi_t' + F_t S_W F_t'."""
    N = int(sc["N"])
    nx, nu = np.asarray(B_list[0]).shape
    sw = np.tile(np.diag(sc["W"]), N)           # diagonal of S_W = blkdiag(W, ..., W)
    F = np.zeros((nx, N * nx))
    Phi = np.eye(nx)
    total = 0.0
    for t in range(N + 1):
        Qt = sc["QN"] if t == N else sc["Q"]
        Sig = Phi @ sc["Sigma0"] @ Phi.T + (F * sw) @ F.T
        total += float(mu[t] @ Qt @ mu[t]) + float(np.sum(Qt * Sig))
        if t == N:
            break
        Kt = K[t * nu:(t + 1) * nu]
        total += float(v[t] @ sc["R"] @ v[t]) + float(np.sum(sc["R"] * ((Kt * sw) @ Kt.T)))
        F = A_list[t] @ F + B_list[t] @ Kt
        F[:, t * nx:(t + 1) * nx] += np.eye(nx)
        Phi = A_list[t] @ Phi
    return total


@dataclass
class ScpRecord:
    """One outer iteration of one scenario."""
    inner: int            # COSMO steps of the convex solve (-1: budget reached)
    rho: float            # trust radius the convex program used
    phi_ref: float        # merit at the reference
    phi_new: float        # merit at the candidate
    model: float          # the convex program's objective at its solution
    ratio: float          # actual / predicted decrease (nan when nothing was predicted)
    defect: float         # max |mu_{t+1} - f(mu_t, v_t)| at the candidate
    nu: float             # max |virtual control|
    accepted: bool


@dataclass
class ScpResult:
    converged: bool
    outer: int               # outer iterations run
    history: List[ScpRecord]
    mu: np.ndarray           # the last accepted reference
    v: np.ndarray
    K: np.ndarray
    inner_total: int = 0     # COSMO steps over all convex solves (a solve stopped by the budget counts it)


@dataclass
class ScpTiming:
    build_s: float = 0.0      # host: linearisation and conic assembly
    upload_s: float = 0.0     # host: super-batch plan and device copies
    solve_s: float = 0.0      # cosmo_solve over the super-batch
    host_s: float = 0.0       # host: merits and ratio tests
    rounds: int = 0
    batch_sizes: List[int] = field(default_factory=list)


class _Scenario:
    def __init__(self, sc, step, jacobians, reference):
        self.sc = sc
        self.N = int(sc["N"])
        self.mu, self.v = (np.array(a, np.float64) for a in reference(sc))
        self.nx, self.nu = self.mu.shape[1], self.v.shape[1]
        self.K = np.zeros((self.N * self.nu, self.N * self.nx))
        self.step, self.jacobians = step, jacobians
        self.A, self.B = self.linearise(self.mu, self.v)
        self.phi = self.merit(self.mu, self.v, self.K, self.A, self.B)
        self.rho = float(sc["rho_x"])
        self.history: List[ScpRecord] = []
        self.converged = False
        self.done = False

    def linearise(self, mu, v):
        AB = [self.jacobians(mu[t], v[t]) for t in range(self.N)]
        return [np.asarray(a) for a, _ in AB], [np.asarray(b) for _, b in AB]

    def defect(self, mu, v):
        return np.stack([mu[t + 1] - self.step(mu[t], v[t]) for t in range(self.N)])

    def merit(self, mu, v, K, A, B):
        return expected_cost(self.sc, A, B, mu, v, K) + self.sc["lam_nu"] * float(np.abs(self.defect(mu, v)).sum())


def scp_solve(scenarios: Sequence[dict], *, step: Callable, jacobians: Callable, subproblem: Callable,
              unpack: Callable, reference: Callable, eps: float = 1e-6, max_outer: int = 30, tol: float = 1e-3,
              eta=(0.0, 0.25, 0.75), shrink: float = 0.5, expand: float = 2.0, inner_max: int = 100000,
              check: int = 1, dtype=torch.float64, device="cuda:0", cg_tol=None, timing: ScpTiming = None,
              progress: Callable = None, **solve_kw) -> List[ScpResult]:
    """Runs the outer loop for every scenario from its reference (K = 0).
    `eps` is the convex solves' absolute and relative tolerance; `check` the
    number of COSMO steps between their stopping tests (1: exact counts);
    further keywords go to `CosmoBatch.solve`.  Returns one ScpResult per
    scenario; `timing`, when given, collects where the time went, and
    `progress(round, scenarios_running, seconds, inner_steps)` is called
    after each outer iteration (inner_steps: the convex solves' step counts,
    -1 where the budget ran out)."""
    if check < 1:
        raise ValueError("check must be >= 1")
    tm = timing if timing is not None else ScpTiming()
    runs = [_Scenario(sc, step, jacobians, reference) for sc in scenarios]
    for _ in range(max_outer):
        active = [r for r in runs if not r.done]
        if not active:
            break
        t0 = time.perf_counter()
        insts = [subproblem(r.sc, r.mu, r.v, r.rho, r.rho) for r in active]
        t1 = time.perf_counter()
        batch = CosmoBatch(insts, K=check, dtype=dtype, device=device, cg_tol=cg_tol, cg_max_iter=2000)
        torch.cuda.synchronize(batch.device)
        t2 = time.perf_counter()
        iters, _, x, _, _ = batch.solve(eps_abs=eps, eps_rel=eps, max_iter=inner_max, **solve_kw)
        xs = x.double().cpu().numpy()
        t3 = time.perf_counter()
        for i, (r, inst) in enumerate(zip(active, insts)):
            mu, v, K, vn = (np.asarray(a, np.float64) for a in
                            unpack(inst, xs[batch.n_off[i]:batch.n_off[i + 1]]))
            model = expected_cost(r.sc, r.A, r.B, mu, v, K) + r.sc["lam_nu"] * float(np.abs(vn).sum())
            A_n, B_n = r.linearise(mu, v)
            d = r.defect(mu, v)
            phi_new = expected_cost(r.sc, A_n, B_n, mu, v, K) + r.sc["lam_nu"] * float(np.abs(d).sum())
            predicted, actual = r.phi - model, r.phi - phi_new
            ratio = actual / predicted if predicted > 0 else float("nan")
            rec = ScpRecord(inner=int(iters[i]), rho=r.rho, phi_ref=r.phi, phi_new=phi_new, model=model, ratio=ratio,
                            defect=float(np.abs(d).max()), nu=float(np.abs(vn).max()), accepted=False)
            r.history.append(rec)
            if not predicted > 1e-12 * abs(r.phi):     # the model predicts no decrease: stationary
                r.done = True
                continue
            if ratio >= eta[0]:
                rec.accepted = True
                r.mu, r.v, r.K, r.A, r.B, r.phi = mu, v, K, A_n, B_n, phi_new
                if rec.defect < tol and rec.nu < tol:
                    r.converged = r.done = True
                    continue
            if ratio < eta[1]:
                r.rho *= shrink
            elif ratio > eta[2]:
                r.rho *= expand
        batch.close()
        t4 = time.perf_counter()
        tm.build_s += t1 - t0
        tm.upload_s += t2 - t1
        tm.solve_s += t3 - t2
        tm.host_s += t4 - t3
        tm.rounds += 1
        tm.batch_sizes.append(len(active))
        if progress is not None:
            progress(tm.rounds, len(active), t4 - t0, np.asarray(iters))
    # steps actually run: a solve that stopped at the budget ran the budget's
    # last multiple of the check interval
    spent = lambda h: h.inner if h.inner >= 0 else inner_max // check * check
    return [ScpResult(converged=r.converged, outer=len(r.history), history=r.history, mu=r.mu, v=r.v, K=r.K,
                      inner_total=int(sum(spent(h) for h in r.history))) for r in runs]
