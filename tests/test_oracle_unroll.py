"""Pins of the oracle's COSMO step, reverse mode and loss (CPU only).

What fixes each part independently of the oracle's own formulas:
  * the reduced solve against the full saddle-point system eq:cosmo_linear_system;
  * gradients against central finite differences;
  * per-step Moreau invariants (y+ in the polar cone, complementarity);
  * a known KKT point that must be a fixed point for every (rho, alpha);
  * converged objective values against closed forms / an independent LP.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import oracle
import synth
from oracle.cosmo import run_fixed

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mixed(seed=7):
    rng = np.random.default_rng(seed)
    return synth.random_mixed(rng), rng


def test_reduced_solve_equals_full_saddle_system():
    inst, rng = _mixed(3)
    n, m = inst.n, inst.m
    x, s, y = rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(m)
    rho = rng.uniform(0.1, 2.0, m)
    st = oracle.step_forward(inst, x, s, y, rho, 1.6)
    rh = st["rho_hat"]
    sigma = 1e-6
    K = np.block([[inst.P.toarray() + sigma * np.eye(n), inst.A.toarray().T],
                  [inst.A.toarray(), -np.diag(1.0 / rh)]])
    rhs = np.concatenate([sigma * x - inst.q, inst.b - s + y / rh])
    sol = np.linalg.solve(K, rhs)
    xt, nu = sol[:n], sol[n:]
    assert np.allclose(st["xt"], xt, atol=1e-9, rtol=1e-9)
    assert np.allclose(st["st"], s - (y + nu) / rh, atol=1e-9, rtol=1e-9)


def test_unroll_gradients_match_finite_differences_mixed_cones():
    inst, rng = _mixed(7)
    K = 6
    rho, alpha = synth.perturbed_hyper(inst, K, rng)
    z = [0.3 * rng.standard_normal(d) for d in (inst.n, inst.m, inst.m)]
    res = oracle.fd_check_unroll(inst, rho, alpha, *z, rng, ndirs=3)
    assert len(res) >= 12
    for g, a, f in res:
        assert abs(a - f) <= 2e-6 * max(1.0, abs(f)), (g, a, f)


def test_unroll_gradients_match_finite_differences_maxcut():
    rng = np.random.default_rng(17)
    inst = synth.maxcut_sdp(5, synth.erdos_renyi(5, 0.6, rng))
    K = 8
    rho, alpha = synth.perturbed_hyper(inst, K, rng)
    res = oracle.fd_check_unroll(inst, rho, alpha, None, None, None, rng, ndirs=3,
                                 groups=("rho", "alpha"))
    assert len(res) >= 4
    for g, a, f in res:
        assert abs(a - f) <= 2e-6 * max(1.0, abs(f)), (g, a, f)


def test_implicit_solve_vjp_matches_fd_appb():
    # App. B sampler (diagonal P, 1%-style sparse A, rho ~ U(0,1)), loss 1/2||x - x*||^2
    rng = np.random.default_rng(4)
    P, A, rho, b, xstar = synth.appb_instance(80, rng, density=0.1)
    q = rng.standard_normal(80)

    class Inst:
        pass
    inst = Inst()
    inst.P, inst.A = P, A
    xi = A.T @ b - q

    def xt_of(r):
        return oracle.solve_reduced(inst, r, 1e-6).solve(xi)
    xt = xt_of(rho)
    lu = oracle.solve_reduced(inst, rho, 1e-6)
    _, g = oracle.implicit_solve_vjp(lu, A, xt, xt - xstar)
    for _ in range(5):
        d = rng.standard_normal(len(rho)) * rho
        h = 1e-6
        fp = 0.5 * np.sum((xt_of(rho + h * d) - xstar) ** 2)
        fm = 0.5 * np.sum((xt_of(rho - h * d) - xstar) ** 2)
        fd = (fp - fm) / (2 * h)
        assert abs(g @ d - fd) <= 1e-6 * max(1.0, abs(fd))


def test_residual_loss_gradient_matches_fd():
    inst, rng = _mixed(5)
    z = [rng.standard_normal(d) for d in (inst.n, inst.m, inst.m)]
    gr = oracle.residual_loss_grad(inst, *z)
    for i in range(3):
        d = rng.standard_normal(len(z[i]))
        zp = list(z); zm = list(z)
        zp[i] = z[i] + 1e-6 * d; zm[i] = z[i] - 1e-6 * d
        fd = (oracle.residual_loss(inst, *zp) - oracle.residual_loss(inst, *zm)) / 2e-6
        assert abs(gr[i] @ d - fd) <= 1e-6 * max(1.0, abs(fd))


def _polar_and_complementarity(inst, s, y):
    for c, sl in synth.cone_row_slices(inst.cones):
        sb, yb = s[sl], y[sl]
        assert abs(sb @ yb) <= 1e-9 * max(1.0, np.linalg.norm(sb) * np.linalg.norm(yb))
        if c.kind == "nonneg":
            assert np.all(yb <= 1e-12)
        elif c.kind == "soc":
            assert np.linalg.norm(yb[1:]) <= -yb[0] + 1e-10      # -y in SOC
        elif c.kind == "psd":
            assert np.linalg.eigvalsh(oracle.smat(yb)).max() <= 1e-10


def test_every_step_keeps_y_in_polar_cone_and_complementary():
    inst, rng = _mixed(11)
    K = 10
    rho, alpha = synth.perturbed_hyper(inst, K, rng)
    tape, (xK, sK, yK) = oracle.unroll_forward(inst, rho, alpha)
    for st in tape:
        _polar_and_complementarity(inst, st["sn"], st["yn"])
    inst2 = synth.c2_batch(B=1, p_lo=12, p_hi=12)[0]
    tape, _ = oracle.unroll_forward(inst2, synth.default_rho(inst2, 10), np.full(10, 1.6))
    for st in tape:
        _polar_and_complementarity(inst2, st["sn"], st["yn"])


@pytest.mark.parametrize("n", [4, 7])
def test_kn_maxcut_kkt_point_is_fixed(n):
    inst = synth.maxcut_sdp(n, synth.complete_graph(n))
    J = np.ones((n, n))
    xs = oracle.svec(n / (n - 1) * np.eye(n) - J / (n - 1))
    s = np.concatenate([np.zeros(n), xs])
    y = np.concatenate([-(n / 4) * np.ones(n), -oracle.svec(J) / 4])
    rng = np.random.default_rng(n)
    for _ in range(4):
        rho = rng.uniform(0.01, 10.0, inst.m)
        st = oracle.step_forward(inst, xs, s, y, rho, float(rng.uniform(0.2, 1.9)))
        assert np.allclose(st["xn"], xs, atol=1e-9)
        assert np.allclose(st["sn"], s, atol=1e-9)
        assert np.allclose(st["yn"], y, atol=1e-9)


def _build(entry):
    n = entry["n"]
    g = {"cycle": synth.cycle_graph, "complete": synth.complete_graph}.get(entry["graph"])
    edges = synth.petersen_graph() if entry["graph"] == "petersen" else g(n)
    return synth.lovasz_theta_sdp(n, edges) if entry["problem"] == "lovasz" else synth.maxcut_sdp(n, edges)


def _converged_value(inst, iters=3000):
    x, s, y = run_fixed(inst, synth.default_rho(inst, 1)[0], 1.6, iters)
    rp, rd = oracle.kkt_residuals(inst, x, s, y)
    return -float(inst.q @ x), float(np.linalg.norm(rp)), float(np.linalg.norm(rd))


@pytest.mark.parametrize("entry", json.load(open(os.path.join(GOLD, "closed_forms.json")))["entries"],
                         ids=lambda e: e["name"])
def test_converged_value_matches_closed_form(entry):
    val, rp, rd = _converged_value(_build(entry))
    assert abs(val - entry["value"]) < 1e-8, (val, entry["value"])
    assert rp < 1e-8 and rd < 1e-8


def _circulant_theta_lp(n, S):
    # X circulant symmetric: c_k = c_{n-k}; theta = max n*mu_0 s.t. n c_0 = 1,
    # c_d = 0 for d in S, mu_j = sum_k c_k cos(2 pi j k / n) >= 0 for all j.
    ks = [k for k in range(0, n // 2 + 1) if k not in S]
    def mult(k):
        return 1.0 if (k == 0 or (n % 2 == 0 and k == n // 2)) else 2.0
    M = np.array([[mult(k) * math.cos(2 * math.pi * j * k / n) for k in ks] for j in range(n)])
    c = -n * M[0]
    res = linprog(c, A_ub=-M, b_ub=np.zeros(n), A_eq=np.array([[n * (k == 0) for k in ks]]),
                  b_eq=[1.0], bounds=[(None, None)] * len(ks), method="highs")
    return -res.fun


@pytest.mark.parametrize("n,S", [(10, [1, 3]), (12, [2, 5]), (13, [1, 4])])
def test_circulant_theta_matches_lp_and_complement_product(n, S):
    G = synth.circulant(n, S)
    Sc = [d for d in range(1, n // 2 + 1) if d not in S]
    th, rp, rd = _converged_value(synth.lovasz_theta_sdp(n, G), 4000)
    thc, _, _ = _converged_value(synth.lovasz_theta_sdp(n, synth.circulant(n, Sc)), 4000)
    assert abs(th - _circulant_theta_lp(n, S)) < 1e-6
    assert abs(th * thc - n) < 1e-5          # theta(G) theta(complement) = n (vertex-transitive)


def test_c1_sdp_brackets_brute_force_maxcut():
    inst = synth.c1_instance()
    edges = inst.meta["edges"]
    val, rp, rd = _converged_value(inst, 4000)
    assert rp < 1e-7 and rd < 1e-7
    n = 20
    # brute force over cuts with vertex 0 fixed on one side
    bits = ((np.arange(2 ** (n - 1))[:, None] >> np.arange(n - 1)) & 1).astype(np.int8)
    side = np.concatenate([np.zeros((len(bits), 1), np.int8), bits], axis=1)
    e = np.array(edges)
    cut = np.zeros(len(side), np.int32)
    for i, j in e:
        cut += side[:, i] != side[:, j]
    best = int(cut.max())
    assert best - 1e-9 <= val <= best / 0.87856 + 1e-9


def test_table2_defaults_drive_default_rho():
    t2 = json.load(open(os.path.join(GOLD, "table2_defaults.json")))
    inst, _ = _mixed(1)
    r = synth.default_rho(inst, 2)
    for c, sl in synth.cone_row_slices(inst.cones):
        assert np.allclose(r[:, sl], t2["rho_init"][c.kind])
    assert t2["alpha_init"] == 1.6 and t2["sigma"] == oracle.Hyper().sigma


def test_stored_precision_rounding_option():
    """unroll_forward(store_dtype=...) rounds what a pipeline of that
    precision stores, nothing else: float64 leaves the run bit for bit as it
    is; float32 leaves every stored per-step value (and the PSD eigenpairs of
    the reverse pass) a float32 number, keeps the float64 right-hand side,
    and on a contractive instance moves the iterates by no more than the
    rounding of K steps."""
    inst, rng = _mixed(13)
    K = 8
    rho, alpha = synth.perturbed_hyper(inst, K, rng)
    rho, alpha = rho.astype(np.float32).astype(np.float64), alpha.astype(np.float32).astype(np.float64)
    tape, z = oracle.unroll_forward(inst, rho, alpha)
    tape64, z64 = oracle.unroll_forward(inst, rho, alpha, store_dtype=np.float64)
    for a, b in zip(z, z64):
        assert np.array_equal(a, b)
    for st, st64 in zip(tape, tape64):
        for key in ("xt", "st", "xn", "sh", "v", "sn", "yn", "xi"):
            assert np.array_equal(st[key], st64[key])
    tape32, z32 = oracle.unroll_forward(inst, rho, alpha, store_dtype=np.float32)
    is32 = lambda a: np.array_equal(np.asarray(a).astype(np.float32).astype(np.float64), a)
    for st in tape32:
        for key in ("rho_hat", "xt", "st", "xn", "sh", "v", "sn", "yn"):
            assert is32(st[key]), key
        assert not is32(st["xi"])          # formed and used in float64, never stored
        for a in st["aux"]:
            if a is not None:
                assert is32(a[0]) and is32(a[1])
    # max-cut on K_6 from z0 = 0 with the default penalties contracts toward its
    # KKT point: the rounded run stays within K float32 roundings of the exact one
    inst2 = synth.maxcut_sdp(6, synth.complete_graph(6))
    r2 = synth.default_rho(inst2, 30)
    _, za = oracle.unroll_forward(inst2, r2, np.full(30, 1.6))
    _, zb = oracle.unroll_forward(inst2, r2, np.full(30, 1.6), store_dtype=np.float32)
    for a, b in zip(za, zb):
        assert 0 < np.linalg.norm(a - b) <= 30 * 6e-8 * 10 * np.linalg.norm(a)


def test_rounding_model_dither_and_solve_residual():
    """The rounding model's realisations: dithered stored values stay float32
    numbers within one unit in the last place of the nearest rounding, and a
    modelled solve residual is what was asked for."""
    inst, rng = _mixed(17)
    K = 5
    rho, alpha = synth.perturbed_hyper(inst, K, rng)
    tape_n, _ = oracle.unroll_forward(inst, rho, alpha, store_dtype=np.float32)
    tape_d, _ = oracle.unroll_forward(inst, rho, alpha, store_dtype=np.float32,
                                      store_rng=np.random.default_rng(3))
    # rho_hat, the first stored value of step 0, comes from the same input in
    # both runs: the two differ by the dither alone
    a, b = tape_n[0]["rho_hat"], tape_d[0]["rho_hat"]
    ulp = np.abs(np.spacing(a.astype(np.float32))).astype(np.float64)
    assert np.all(np.abs(a - b) <= ulp * 1.0000001) and np.any(a != b)
    for st in tape_d:
        for key in ("rho_hat", "xt", "st", "xn", "sh", "v", "sn", "yn"):
            assert np.array_equal(st[key].astype(np.float32).astype(np.float64), st[key]), key
    tape_r, _ = oracle.unroll_forward(inst, rho, alpha, store_dtype=np.float32,
                                      store_rng=np.random.default_rng(4), solve_resid=1e-3)
    st = tape_r[0]
    M = oracle.reduced_matrix(inst, st["rho_hat"], 1e-6)
    res = np.linalg.norm(M @ st["xt"] - st["xi"]) / np.linalg.norm(st["xi"])
    assert 0.5e-3 < res < 2e-3          # 1e-3 up to the float32 rounding of x~


# ---- the vanilla baseline: COSMO to tolerance with residual balancing ----------

def _stop_ok(inst, x, s, y, eps_abs, eps_rel):
    rp, rd = oracle.kkt_residuals(inst, x, s, y)
    Np = max(np.abs(inst.A @ x).max(), np.abs(s).max(), np.abs(inst.b).max())
    Nd = max(np.abs(inst.P @ x).max(), np.abs(inst.q).max(), np.abs(inst.A.T @ y).max())
    return np.abs(rp).max() <= eps_abs + eps_rel * Np and np.abs(rd).max() <= eps_abs + eps_rel * Nd


@pytest.mark.parametrize("entry", json.load(open(os.path.join(GOLD, "closed_forms.json")))["entries"],
                         ids=lambda e: e["name"])
def test_residual_balancing_stops_at_the_first_passing_iterate(entry):
    """The returned count is the first iterate that meets the stopping test;
    the value there is the closed form to within the tolerance's reach."""
    inst = _build(entry)
    k, (x, s, y), rho = oracle.solve_residual_balancing(inst)
    assert k is not None and _stop_ok(inst, x, s, y, 1e-3, 1e-3)
    k1, (x1, s1, y1), _ = oracle.solve_residual_balancing(inst, max_iter=k - 1)
    assert k1 is None and not _stop_ok(inst, x1, s1, y1, 1e-3, 1e-3)
    assert abs(-float(inst.q @ x) - entry["value"]) <= 3e-2 * entry["value"]


def test_residual_balancing_without_updates_is_fixed_penalty_cosmo():
    inst = _build({"problem": "lovasz", "graph": "petersen", "n": 10})
    k, (x, s, y), rho = oracle.solve_residual_balancing(inst, adapt=False)
    assert rho == 0.1
    xf, sf, yf = run_fixed(inst, synth.default_rho(inst, 1)[0], 1.6, k)
    assert np.allclose(x, xf, rtol=0, atol=1e-12) and np.allclose(y, yf, rtol=0, atol=1e-12)


@pytest.mark.parametrize("c", [1e-2, 30.0])
def test_residual_balancing_is_invariant_to_cost_scaling(c):
    """Scaling P, q (and sigma, rho) by c scales y and r_d by c and leaves x,
    s and the normalised residuals unchanged, so with relative tolerances the
    same steps are taken, the updates happen at the same steps and the final
    penalty is c times the unscaled one.  A rule that dropped a normaliser
    or the square root would break this."""
    import copy
    inst = _build({"problem": "lovasz", "graph": "cycle", "n": 7})
    k, (x, s, y), rho = oracle.solve_residual_balancing(inst, eps_abs=0.0)
    assert rho != 0.1                      # the rule fired
    sc = copy.copy(inst)
    sc.P, sc.q = inst.P * c, inst.q * c
    kc, (xc, sc_, yc), rhoc = oracle.solve_residual_balancing(sc, rho0=0.1 * c, eps_abs=0.0, sigma=1e-6 * c,
                                                              rho_min=1e-6 * c, rho_max=1e6 * c)
    assert kc == k
    assert rhoc == pytest.approx(c * rho, rel=1e-9)
    assert np.allclose(xc, x, rtol=1e-7, atol=1e-9) and np.allclose(yc, c * y, rtol=1e-7, atol=1e-9 * c)


# ---- SCP for nonlinear covariance steering (App. F) ------------------------------

def _unicycle_scp(seed, N=4, **kw):
    from oracle.scp import scp
    from synth.covsteer import (unicycle_scenario, unicycle_subproblem, unicycle_initial_reference, unicycle_step,
                                unicycle_jacobians, unpack_solution)
    sc = unicycle_scenario(np.random.default_rng(seed), N=N)
    mu0, v0 = unicycle_initial_reference(sc)
    out = scp(sc, lambda x, u: unicycle_step(x, u, sc["dt"]), lambda x, u: unicycle_jacobians(x, u, sc["dt"]),
              unicycle_subproblem, unpack_solution, mu0, v0, **kw)
    return sc, out


def test_scp_on_linear_dynamics_converges_in_one_step():
    """App. F: with linear dynamics (the double integrator) the SCP loop
    converges in a single iteration -- the linearisation is exact, so the
    first convex step has no defect and the ratio is one."""
    from oracle.scp import scp
    from synth.covsteer import covsteer_ltv, unpack_solution
    dt, N = 0.5, 5
    I2 = np.eye(2)
    A = np.block([[I2, dt * I2], [np.zeros((2, 2)), I2]])
    B = np.vstack([0.5 * dt * dt * I2, dt * I2])
    Q = np.diag([1.0, 1.0, 0.3, 0.3])
    sc = dict(N=N, W=np.diag([dt ** 3 / 3 * 0.09] * 2 + [dt * 0.09] * 2), Sigma0=1e-4 * np.eye(4), sigma_N=0.25,
              Q=Q, R=0.1 * np.eye(2), QN=10 * Q, lam_nu=100.0, rho_x=5.0, mu0=np.zeros(4),
              goal=np.array([2.0, -1.0, 0.0, 0.0]))

    def sub(sc, mu_r, v_r, rx, ru):
        return covsteer_ltv([A] * N, [B] * N, [np.zeros(4)] * N, sc["W"], sc["mu0"], sc["goal"], sc["Sigma0"],
                            sc["sigma_N"], sc["Q"], sc["R"], sc["QN"], sc["lam_nu"], trust=(mu_r, v_r, rx, ru))

    lam = np.linspace(0, 1, N + 1)[:, None]
    out = scp(sc, lambda x, u: A @ x + B @ u, lambda x, u: (A, B), sub, unpack_solution,
              sc["goal"][None, :] * lam, np.zeros((N, 2)), eps=1e-9)
    assert out["converged"] and out["outer"] == 1
    h = out["history"][0]
    assert h["ratio"] == pytest.approx(1.0, abs=1e-6) and h["defect"] < 1e-6


def test_scp_unicycle_converges_with_monotone_merit():
    """The accepted merits decrease, the radius follows the ratio rule, and
    the final trajectory meets the stopping test on the nonlinear dynamics."""
    from synth.covsteer import unicycle_step
    sc, out = _unicycle_scp(1, N=4)
    assert out["converged"]
    acc = [h for h in out["history"] if h["accepted"]]
    merits = [acc[0]["phi_ref"]] + [h["phi_new"] for h in acc]
    assert all(b < a for a, b in zip(merits, merits[1:]))
    for h0, h1 in zip(out["history"], out["history"][1:]):
        r = h0["ratio"]
        expect = h0["rho"] * (0.5 if r < 0.25 else (2.0 if r > 0.75 else 1.0))
        assert h1["rho"] == pytest.approx(expect)
    mu, v = out["mu"], out["v"]
    d = np.array([mu[t + 1] - unicycle_step(mu[t], v[t], sc["dt"]) for t in range(sc["N"])])
    assert np.abs(d).max() < 1e-3
    assert np.allclose(mu[0], sc["mu0"], atol=1e-4) and np.allclose(mu[-1], sc["goal"], atol=1e-4)
