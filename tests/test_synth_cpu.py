"""The double-integrator covariance-steering generator against the problem it
encodes (App. F, "Covariance Steering"): the PSD rows are the terminal
Schur-complement LMI of the closed-loop covariance, and 0.5 x'Px + q'x is the
mean-plus-covariance cost up to a constant.  Both sides are written here
from the dynamics directly (stacked rollout matrices, traces), not from the
generator's sparse assembly."""
import numpy as np

import synth
from oracle.svec import smat


def _unpack_k(inst, x):
    """The strictly block lower-triangular feedback gain K (N nu x N nx) from x."""
    md = inst.meta
    N, nx, nu = md["N"], md["nx"], md["nu"]
    K = np.zeros((N * nu, N * nx))
    idx = md["k_base"]
    for t in range(N):
        for tau in range(t):
            K[t * nu:(t + 1) * nu, tau * nx:(tau + 1) * nx] = x[idx:idx + nu * nx].reshape(nu, nx)
            idx += nu * nx
    assert idx == md["k_base"] + md["nk"]
    return K


def _rollout(A, B, t, N, nx, nu):
    """Bbar_t, Dbar_t: x_t = A^t x_0 + Bbar_t U + Dbar_t W over the first t steps."""
    Bb, Db = np.zeros((nx, N * nu)), np.zeros((nx, N * nx))
    for tp in range(t):
        Ap = np.linalg.matrix_power(A, t - 1 - tp)
        Bb[:, tp * nu:(tp + 1) * nu] = Ap @ B
        Db[:, tp * nx:(tp + 1) * nx] = Ap
    return Bb, Db


def _direct_cost(inst, x):
    md = inst.meta
    N, nx, nu, A, B, W = md["N"], md["nx"], md["nu"], md["A"], md["B"], md["W"]
    K = _unpack_k(inst, x)
    SW = np.kron(np.eye(N), W)
    Q = np.diag([1.0, 1.0, 0.3, 0.3])
    R = 0.1 * np.eye(nu)
    f = 0.0
    for t in range(N + 1):
        Qt = 10.0 * Q if t == N else Q
        mu = x[t * nx:(t + 1) * nx]
        f += mu @ Qt @ mu
        if t >= 1:
            Bb, Db = _rollout(A, B, t, N, nx, nu)
            F = Db + Bb @ K
            f += np.trace(Qt @ F @ SW @ F.T)
    v0 = (N + 1) * nx
    for t in range(N):
        v = x[v0 + t * nu:v0 + (t + 1) * nu]
        f += v @ R @ v
        Kt = K[t * nu:(t + 1) * nu]
        f += np.trace(R @ Kt @ SW @ Kt.T)
    f += 100.0 * x[-N * nx:].sum()
    return f


def test_double_integrator_lmi_is_the_terminal_covariance_bound():
    rng = np.random.default_rng(0)
    inst = synth.double_integrator_cs(rng)
    md = inst.meta
    N, nx, nu, A, B, W = md["N"], md["nx"], md["nu"], md["A"], md["B"], md["W"]
    assert [c.kind for c in inst.cones] == ["zero", "nonneg", "psd"]
    p = inst.cones[-1].size
    assert p == nx + N * nx
    for _ in range(3):
        x = rng.standard_normal(inst.n)
        K = _unpack_k(inst, x)
        Bb, Db = _rollout(A, B, N, N, nx, nu)
        F = (Db + Bb @ K) @ np.sqrt(np.kron(np.eye(N), W))
        AN = np.linalg.matrix_power(A, N)
        lmi = np.block([[md["sigma_N"] ** 2 * np.eye(nx) - AN @ md["Sigma_0"] @ AN.T, F],
                        [F.T, np.eye(N * nx)]])
        s = inst.b - inst.A @ x
        got = smat(s[-p * (p + 1) // 2:])
        assert np.abs(got - lmi).max() <= 1e-13 * max(1.0, np.abs(lmi).max())
        # Schur complement: the LMI holds iff Sigma_N <= sigma_N^2 I
        SigN = AN @ md["Sigma_0"] @ AN.T + F @ F.T
        assert (np.linalg.eigvalsh(lmi).min() >= -1e-12) == \
            (np.linalg.eigvalsh(md["sigma_N"] ** 2 * np.eye(nx) - SigN).min() >= -1e-12)


def test_double_integrator_cost_matches_the_direct_cost():
    rng = np.random.default_rng(1)
    inst = synth.double_integrator_cs(rng)
    obj = lambda x: 0.5 * x @ (inst.P @ x) + inst.q @ x
    for _ in range(3):
        x, y = rng.standard_normal(inst.n), rng.standard_normal(inst.n)
        d_direct = _direct_cost(inst, x) - _direct_cost(inst, y)
        assert abs((obj(x) - obj(y)) - d_direct) <= 1e-10 * max(1.0, abs(d_direct))


def test_double_integrator_rows_encode_dynamics_and_l1_epigraph():
    rng = np.random.default_rng(2)
    inst = synth.double_integrator_cs(rng)
    md = inst.meta
    N, nx, nu, A, B = md["N"], md["nx"], md["nu"], md["A"], md["B"]
    x = rng.standard_normal(inst.n)
    s = inst.b - inst.A @ x
    mu = x[:(N + 1) * nx].reshape(N + 1, nx)
    v = x[(N + 1) * nx:(N + 1) * nx + N * nu].reshape(N, nu)
    nuv = x[-2 * N * nx:-N * nx].reshape(N, nx)
    e = x[-N * nx:]
    n0, n1 = inst.cones[0].size, inst.cones[1].size
    z = s[:n0]
    # zero-cone slack b - A x is minus the residual of each equality
    assert np.allclose(z[:nx], -mu[0])
    for t in range(N):
        assert np.allclose(z[nx + t * nx:nx + (t + 1) * nx], -(mu[t + 1] - A @ mu[t] - B @ v[t] - nuv[t]))
    assert np.allclose(z[(N + 1) * nx:], md["goal"] - mu[N])
    assert np.allclose(s[n0:n0 + n1], np.concatenate([e - nuv.ravel(), e + nuv.ravel()]))


# ---- the LTV builder with trust regions, and the unicycle ---------------------------

def test_unicycle_jacobians_match_finite_differences():
    from synth.covsteer import unicycle_jacobians, unicycle_step
    rng = np.random.default_rng(3)
    for _ in range(5):
        x, u = rng.standard_normal(3), rng.standard_normal(2)
        A, B = unicycle_jacobians(x, u)
        h = 1e-6
        Afd = np.stack([(unicycle_step(x + h * e, u) - unicycle_step(x - h * e, u)) / (2 * h) for e in np.eye(3)], 1)
        Bfd = np.stack([(unicycle_step(x, u + h * e) - unicycle_step(x, u - h * e)) / (2 * h) for e in np.eye(2)], 1)
        assert np.allclose(A, Afd, atol=1e-8) and np.allclose(B, Bfd, atol=1e-8)


def _ltv_case(rng, N=4, nx=3, nu=2):
    from synth.covsteer import covsteer_ltv
    A = [np.eye(nx) + 0.2 * rng.standard_normal((nx, nx)) for _ in range(N)]
    B = [rng.standard_normal((nx, nu)) for _ in range(N)]
    r = [rng.standard_normal(nx) for _ in range(N)]
    W = np.diag(rng.uniform(0.01, 0.05, nx))
    Q = np.diag(rng.uniform(0.5, 2.0, nx))
    R = np.diag(rng.uniform(0.1, 0.5, nu))
    mu_ref, v_ref = rng.standard_normal((N + 1, nx)), rng.standard_normal((N, nu))
    inst = covsteer_ltv(A, B, r, W, rng.standard_normal(nx), rng.standard_normal(nx), 0.01 * np.eye(nx), 0.5, Q, R,
                        5.0 * Q, 100.0, trust=(mu_ref, v_ref, 2.0, 3.0))
    return inst, A, B, r, W, Q, R, mu_ref, v_ref


def _phi(A, t, tau):
    M = np.eye(A[0].shape[0])
    for s in range(tau, t):
        M = A[s] @ M
    return M


def test_ltv_builder_terminal_lmi_trust_regions_and_dynamics():
    from synth.covsteer import unpack_solution
    rng = np.random.default_rng(4)
    inst, A, B, r, W, Q, R, mu_ref, v_ref = _ltv_case(rng)
    md = inst.meta
    N, nx, nu = md["N"], md["nx"], md["nu"]
    x = rng.standard_normal(inst.n)
    s = inst.b - inst.A @ x
    mu, v, K, vn = unpack_solution(inst, x)
    kinds = [c.kind for c in inst.cones]
    assert kinds == ["zero", "nonneg"] + ["soc"] * (2 * N + 1) + ["psd"]
    n0 = inst.cones[0].size
    for t in range(N):
        assert np.allclose(-s[nx + t * nx:nx + (t + 1) * nx], mu[t + 1] - A[t] @ mu[t] - B[t] @ v[t] - vn[t] - r[t])
    o = n0 + inst.cones[1].size
    for t in range(N + 1):
        assert s[o] == 2.0 and np.allclose(s[o + 1:o + 1 + nx], mu[t] - mu_ref[t])
        o += nx + 1
    for t in range(N):
        assert s[o] == 3.0 and np.allclose(s[o + 1:o + 1 + nu], v[t] - v_ref[t])
        o += nu + 1
    # terminal LMI: x_N's disturbance response (Dbar_N + Bbar_N K) Sigma_W^1/2
    Db = np.hstack([_phi(A, N, tau + 1) for tau in range(N)])
    Bb = np.hstack([_phi(A, N, tau + 1) @ B[tau] for tau in range(N)])
    F = (Db + Bb @ K) @ np.sqrt(np.kron(np.eye(N), W))
    PN = _phi(A, N, 0)
    lmi = np.block([[0.25 * np.eye(nx) - PN @ md["Sigma_0"] @ PN.T, F], [F.T, np.eye(N * nx)]])
    p = nx + N * nx
    assert np.abs(smat(s[-p * (p + 1) // 2:]) - lmi).max() <= 1e-12 * max(1.0, np.abs(lmi).max())


def test_ltv_builder_cost_matches_the_expected_cost():
    from synth.covsteer import unpack_solution
    rng = np.random.default_rng(5)
    inst, A, B, r, W, Q, R, mu_ref, v_ref = _ltv_case(rng)
    md = inst.meta
    N, nx, nu = md["N"], md["nx"], md["nu"]
    SW = np.kron(np.eye(N), W)

    def direct(x):
        mu, v, K, vn = unpack_solution(inst, x)
        f = 0.0
        for t in range(N + 1):
            Qt = 5.0 * Q if t == N else Q
            f += mu[t] @ Qt @ mu[t]
            if t >= 1:
                Db = np.hstack([_phi(A, t, tau + 1) if tau < t else np.zeros((nx, nx)) for tau in range(N)])
                Bb = np.hstack([_phi(A, t, tau + 1) @ B[tau] if tau < t else np.zeros((nx, nu)) for tau in range(N)])
                Ft = Db + Bb @ K
                f += np.trace(Qt @ Ft @ SW @ Ft.T)
        for t in range(N):
            f += v[t] @ R @ v[t]
            Kt = K[t * nu:(t + 1) * nu]
            f += np.trace(R @ Kt @ SW @ Kt.T)
        return f + 100.0 * x[md["e_base"]:].sum()

    obj = lambda x: 0.5 * x @ (inst.P @ x) + inst.q @ x
    for _ in range(3):
        x, y = rng.standard_normal(inst.n), rng.standard_normal(inst.n)
        d = direct(x) - direct(y)
        assert abs((obj(x) - obj(y)) - d) <= 1e-10 * max(1.0, abs(d))


def test_scp_expected_cost_recursion_matches_the_oracle_rollout():
    """The package's SCP merit carries the covariance forward step by step;
    the oracle's sums transition products.  Both are App. F's expected cost."""
    import oracle.scp
    from paper_2606_13825_amd.scp import expected_cost
    from synth.covsteer import unicycle_scenario
    rng = np.random.default_rng(6)
    sc = unicycle_scenario(rng, N=5)
    N = sc["N"]
    A = [np.eye(3) + 0.1 * rng.standard_normal((3, 3)) for _ in range(N)]
    B = [rng.standard_normal((3, 2)) for _ in range(N)]
    mu, v = rng.standard_normal((N + 1, 3)), rng.standard_normal((N, 2))
    K = np.zeros((N * 2, N * 3))
    for t in range(N):
        K[t * 2:(t + 1) * 2, :t * 3] = rng.standard_normal((2, t * 3))
    a = expected_cost(sc, A, B, mu, v, K)
    b = oracle.scp.expected_cost(sc, A, B, mu, v, K)
    assert abs(a - b) <= 1e-12 * abs(b)


def test_lovasz_reduced_matrix_has_three_jacobi_eigenvalues():
    """On a Lovasz theta SDP, A has one trace row plus rows with a single
    entry (edge equalities, the PSD block's -I), and rectification makes the
    penalty uniform within each cone block.  So diag(M)^-1/2 M diag(M)^-1/2
    is the identity off the svec diagonal positions, and on the p diagonal
    positions a multiple of the identity plus a rank-one term along the
    trace row: three distinct eigenvalues (one small of multiplicity p - 1,
    1, one large), so Jacobi-PCG ends in at most three iterations in exact
    arithmetic, while the condition number is large."""
    from oracle.cones import rectify
    from oracle.cosmo import reduced_matrix
    inst = synth.c3_batch(B=1, n_lo=24, n_hi=24, seed=3)[0]
    rho, _ = synth.perturbed_hyper(inst, 1, np.random.default_rng(0), spread=0.5)
    M = reduced_matrix(inst, rectify(rho[0], inst.cones), 1e-6).toarray()
    dm = 1.0 / np.sqrt(np.diag(M))
    ev = np.linalg.eigvalsh(dm[:, None] * M * dm[None, :])
    groups = np.split(ev, np.where(np.diff(ev) > 1e-8 * ev[-1])[0] + 1)
    assert len(groups) == 3
    p = inst.meta["order"]
    # the diagonal positions: p - 1 directions orthogonal to the trace row, and the trace direction
    assert np.isclose(groups[1][0], 1.0) and groups[0].size == p - 1 and groups[2].size == 1
    assert ev[-1] / ev[0] > 1e3   # the trace row: ill-conditioned although only three eigenvalues
