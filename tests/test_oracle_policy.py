"""Pins of the policy oracle (oracle/policy.py: App. E "Policy
Parameterization", the log-residual loss of Sec. "Experiments", Table 2).

* App. E's initialisation (zero last layers) makes the policy COSMO with the
  fixed initial penalties: the unroll must then equal the fixed-penalty
  oracle step for step.
* The squashing maps onto the Table 2 bounds and inverts.
* Feature probes: a policy whose network passes one feature through
  linearly (bias large enough that both ReLUs are the identity on it) moves
  the logit by exactly c times that feature, so each feature is compared
  with the same quantity computed here from the recorded iterates.
* The loss of a constant trajectory is K log 2; the loss the unroll reports
  equals the loss of its own recorded iterates.
* Finite differences of the whole unrolled loss against the reverse pass, in
  every parameter group, in l^0 and in z^0 (denominators held, as the loss
  detaches them).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import policy as pol

K = 4


def _mixed(seed=3):
    rng = np.random.default_rng(seed)
    return rng, synth.random_mixed(rng, n=8, soc_dims=(3, 4), psd_orders=(3, 2))


def test_zero_heads_are_cosmo_with_fixed_initial_penalties():
    rng, inst = _mixed()
    theta = pol.init_params(rng)
    fw = pol.unroll_policy_forward(inst, theta, K)
    rho0 = np.asarray(pol.TABLE2_RHO0)[pol.row_kinds(inst)]
    assert np.allclose(fw["rho"], rho0[None, :], rtol=1e-12, atol=0)
    assert np.allclose(fw["alpha"], pol.TABLE2_ALPHA0, rtol=1e-14)
    tape, (x, s, y) = oracle.unroll_forward(inst, np.tile(rho0, (K, 1)), np.full(K, pol.TABLE2_ALPHA0))
    for k in range(K):
        for key in ("x", "s", "y"):
            assert np.allclose(fw["tape"][k]["step"][key], tape[k][key], rtol=1e-12, atol=1e-13)
    assert np.allclose(fw["x"], x, rtol=1e-12, atol=1e-13) and np.allclose(fw["y"], y, rtol=1e-12, atol=1e-13)


def test_squashing_bounds_and_inverse():
    import torch
    r = np.array([1.5e-3, 0.1, 1.0, 100.0, 999.0])
    assert np.allclose(pol.squash_rho(torch.from_numpy(pol.logit_of_rho(r))).numpy(), r, rtol=1e-12)
    a = np.array([0.01, 1.0, 1.6, 1.99])
    assert np.allclose(pol.squash_alpha(torch.from_numpy(pol.logit_of_alpha(a))).numpy(), a, rtol=1e-12)
    big = torch.tensor([-50.0, 0.0, 50.0], dtype=torch.float64)
    rr = pol.squash_rho(big).numpy()
    assert rr[0] == pytest.approx(pol.RHO_MIN, rel=1e-12) and rr[1] == pytest.approx(1.0, rel=1e-12)
    assert rr[2] == pytest.approx(pol.RHO_MAX, rel=1e-12)
    aa = pol.squash_alpha(big).numpy()
    assert aa[0] == pytest.approx(0.0, abs=1e-20) and aa[1] == 1.0 and aa[2] == pytest.approx(2.0, rel=1e-15)


def _probe_theta(which: str, j: int, c: float, big: float = 1e3):
    """theta whose `which` MLP ('r' or 'a') outputs c * xi_j exactly."""
    theta = pol.init_params(np.random.default_rng(0))
    p = pol.unpack(theta)
    for pre in ("r", "a"):
        for key in ("W1", "b1", "W2", "b2", "w3", "b3"):
            p[pre + key][...] = 0.0
    p[which + "W1"][j, 0] = 1.0
    p[which + "b1"][0] = big
    p[which + "W2"][0, 0] = 1.0
    p[which + "w3"][0] = c
    p[which + "b3"][...] = -c * big
    return theta


def _kkt_np(inst, x, s, y):
    Ax, Aty, Px = inst.A @ x, inst.A.T @ y, inst.P @ x
    rp, rd = Ax + s - inst.b, Px + inst.q - Aty
    Np = max(np.abs(Ax).max(), np.abs(s).max(), np.abs(inst.b).max())
    Nd = max(np.abs(Px).max(), np.abs(inst.q).max(), np.abs(Aty).max())
    return rp / Np, rd / Nd


def _features_from_tape(inst, fw, k):
    """Row features 1..6 and instance features 1..4 at iterate k, from the
    recorded iterates (s^{k-1} and the s~ that made s^k from step k-1)."""
    st = fw["tape"][k]["step"]
    x, s, y = st["x"], st["s"], st["y"]
    rbp, rbd = _kkt_np(inst, x, s, y)
    if k == 0:
        dp = dd = np.zeros_like(s)
    else:
        prev = fw["tape"][k - 1]["step"]
        dp, dd = s - prev["st"], s - prev["s"]
    lg = lambda v: np.log(np.abs(v).max() + pol.EPS)
    rows = {1: s, 2: y, 3: rbp, 4: np.full_like(s, lg(rbd)), 5: dp, 6: dd}
    inst_f = {1: lg(rbp), 2: lg(rbd), 3: lg(dp), 4: lg(dd)}
    return rows, inst_f


@pytest.mark.parametrize("j", [1, 2, 3, 4, 5, 6])
def test_row_feature_probe(j):
    rng, inst = _mixed(4)
    z0 = [0.3 * rng.standard_normal(d) for d in (inst.n, inst.m, inst.m)]
    c = 1e-3
    fw = pol.unroll_policy_forward(inst, _probe_theta("r", j, c), K, *z0)
    ls = [t["l_rho"] for t in fw["tape"]] + [fw["l_rho"]]
    for k in range(K):
        rows, _ = _features_from_tape(inst, fw, k)
        assert np.allclose(ls[k + 1] - ls[k], c * rows[j], rtol=1e-9, atol=1e-12 * c), (j, k)


@pytest.mark.parametrize("j", [1, 2, 3, 4])
def test_instance_feature_probe(j):
    rng, inst = _mixed(5)
    z0 = [0.3 * rng.standard_normal(d) for d in (inst.n, inst.m, inst.m)]
    c = 1e-3
    fw = pol.unroll_policy_forward(inst, _probe_theta("a", j, c), K, *z0)
    la = [t["l_alpha"] for t in fw["tape"]] + [fw["l_alpha"]]
    for k in range(K):
        _, f = _features_from_tape(inst, fw, k)
        assert la[k + 1] - la[k] == pytest.approx(c * f[j], rel=1e-9, abs=1e-12), (j, k)


def test_logit_feature_is_the_previous_logit():
    """Feature 0 of both networks is the current logit: with the network
    passing it through, l^{k+1} = (1 + c) l^k."""
    rng, inst = _mixed(6)
    c = 0.05
    for which, key in (("r", "l_rho"), ("a", "l_alpha")):
        fw = pol.unroll_policy_forward(inst, _probe_theta(which, 0, c), K)
        ls = [np.asarray(t[key]) for t in fw["tape"]] + [np.asarray(fw[key])]
        for k in range(K):
            assert np.allclose(ls[k + 1], (1 + c) * ls[k], rtol=1e-12)


def test_loss_of_constant_trajectory_and_of_recorded_iterates():
    rng, inst = _mixed(7)
    z = [0.3 * rng.standard_normal(d) for d in (inst.n, inst.m, inst.m)]
    assert pol.log_residual_loss(inst, [z] * (K + 1)) == pytest.approx(K * np.log(2.0), rel=1e-14)
    theta = pol.init_params(rng, head_scale=0.2)
    fw = pol.unroll_policy_forward(inst, theta, K, *z)
    zs = [tuple(t["step"][k] for k in ("x", "s", "y")) for t in fw["tape"]] + [(fw["x"], fw["s"], fw["y"])]
    assert fw["loss"] == pytest.approx(pol.log_residual_loss(inst, zs), rel=1e-13)


def _groups():
    sizes = [("rW1", pol.N_FEAT_RHO * 32), ("rb1", 32), ("rW2", 1024), ("rb2", 32), ("rw3", 32), ("rb3", 1),
             ("aW1", pol.N_FEAT_ALPHA * 32), ("ab1", 32), ("aW2", 1024), ("ab2", 32), ("aw3", 32), ("ab3", 1),
             ("l_rho0", 4), ("l_alpha0", 1)]
    out, o = [], 0
    for nm, cnt in sizes:
        out.append((nm, slice(o, o + cnt)))
        o += cnt
    assert o == pol.PARAM_COUNT
    return out


@pytest.mark.parametrize("family", ["mixed", "maxcut"])
def test_unrolled_loss_gradients_match_finite_differences(family):
    if family == "mixed":
        rng, inst = _mixed(8)
    else:
        rng = np.random.default_rng(9)
        inst = synth.maxcut_sdp(6, synth.erdos_renyi(6, 0.5, rng))
    theta = pol.init_params(rng, head_scale=0.3)
    z0 = [0.5 * rng.standard_normal(d) for d in (inst.n, inst.m, inst.m)]
    fw = pol.unroll_policy_forward(inst, theta, K, *z0)
    bw = pol.unroll_policy_backward(inst, theta, fw)
    D = (fw["Dd"], fw["Dp"])

    def L(th, zz):
        return pol.unroll_policy_forward(inst, th, K, *zz, denominators=D)["loss"]

    h = 1e-6
    for nm, sl in _groups():
        d = np.zeros_like(theta)
        d[sl] = rng.standard_normal(sl.stop - sl.start)
        fd = (L(theta + h * d, z0) - L(theta - h * d, z0)) / (2 * h)
        an = float(bw["g_theta"] @ d)
        assert abs(fd - an) <= 2e-6 * max(abs(fd), 1e-3 * np.linalg.norm(bw["g_theta"])), (nm, fd, an)
    for i, nm in enumerate(("x0", "s0", "y0")):
        dv = rng.standard_normal(z0[i].size)
        zp, zm = list(z0), list(z0)
        zp[i], zm[i] = z0[i] + h * dv, z0[i] - h * dv
        fd = (L(theta, zp) - L(theta, zm)) / (2 * h)
        an = float(bw["g" + nm] @ dv)
        assert abs(fd - an) <= 1e-5 * max(abs(fd), 1e-2), (nm, fd, an)


def test_package_initialiser_follows_the_documented_layout():
    """The package's policy_init and the oracle read the same flat layout:
    zero last layers, Table 2's penalties and relaxation at l^0."""
    import torch
    from paper_2606_13825_amd.binding import policy_init
    th = policy_init(0, 0.0, torch.float64, "cpu").numpy()
    assert th.size == pol.PARAM_COUNT
    p = pol.unpack(th)
    for key in ("rw3", "rb3", "aw3", "ab3"):
        assert np.all(p[key] == 0.0)
    rho0 = pol.squash_rho(torch.from_numpy(np.array(p["l_rho0"]))).numpy()
    assert np.allclose(rho0, pol.TABLE2_RHO0, rtol=1e-12)
    a0 = float(pol.squash_alpha(torch.tensor(float(p["l_alpha0"]), dtype=torch.float64)))
    assert a0 == pytest.approx(pol.TABLE2_ALPHA0, rel=1e-14)
    th2 = policy_init(0, 0.1, torch.float64, "cpu").numpy()
    assert np.abs(pol.unpack(th2)["rw3"]).max() > 0
