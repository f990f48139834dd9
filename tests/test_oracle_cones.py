"""Pins of the oracle's encodings, projections and their VJPs against
mathematics that does not go through the oracle's own formulas (CPU only)."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import appc_matrix, random_orthogonal


def _sym(rng, p):
    G = rng.standard_normal((p, p))
    return 0.5 * (G + G.T)


# --- svec -------------------------------------------------------------------

def test_svec_is_isometry_and_inverse():
    rng = np.random.default_rng(0)
    for p in (1, 2, 5, 9):
        X, Y = _sym(rng, p), _sym(rng, p)
        assert np.isclose(oracle.svec(X) @ oracle.svec(Y), np.trace(X @ Y), rtol=1e-13, atol=1e-13)
        assert np.allclose(oracle.smat(oracle.svec(X)), X, atol=1e-15)
        assert len(oracle.svec(X)) == p * (p + 1) // 2


def test_svec_layout_matches_generator_index():
    # entry (i, j) of a symmetric matrix sits at the generator's svec_index
    p = 6
    X = np.zeros((p, p))
    X[1, 4] = X[4, 1] = 1.0
    v = oracle.svec(X)
    assert np.flatnonzero(v).tolist() == [synth.svec_index(1, 4)]
    assert math.isclose(v[synth.svec_index(1, 4)], math.sqrt(2.0))


# --- PSD projection -----------------------------------------------------------

def _psd_via_svd(S):
    # (S + |S|)/2 with |S| = V diag(sv) V' from the SVD S = U diag(sv) V'
    _, sv, Vt = np.linalg.svd(S)
    return 0.5 * (S + (Vt.T * sv) @ Vt)


def _newton_schulz_sign(S, iters=60):
    # eq:newton-schulz, S_0 = S/||S||_F ; converges for nonsingular S
    X = S / np.linalg.norm(S)
    I = np.eye(len(S))
    for _ in range(iters):
        X = 0.5 * X @ (3.0 * I - X @ X)
    return X


@pytest.mark.parametrize("p", [1, 2, 3, 7, 20, 40])
def test_proj_psd_matches_svd_route_and_moreau(p):
    rng = np.random.default_rng(p)
    S = _sym(rng, p)
    out, U, lam = oracle.proj_psd(oracle.svec(S))
    Pi = oracle.smat(out)
    assert np.allclose(Pi, _psd_via_svd(S), atol=1e-12)
    # Moreau: Pi >= 0, Pi - S >= 0, <Pi, Pi - S> = 0
    assert np.linalg.eigvalsh(Pi).min() > -1e-12
    assert np.linalg.eigvalsh(Pi - S).min() > -1e-12
    assert abs(np.sum(Pi * (Pi - S))) < 1e-11


def test_proj_psd_matches_newton_schulz_small():
    rng = np.random.default_rng(11)
    for p in (2, 4, 6):
        Q = random_orthogonal(p, rng)
        lam = rng.uniform(0.2, 1.0, p) * rng.choice([-1.0, 1.0], p)
        S = (Q * lam) @ Q.T
        Pi = oracle.smat(oracle.proj_psd(oracle.svec(S))[0])
        ns = 0.5 * (S + _newton_schulz_sign(S) @ S)
        assert np.allclose(Pi, ns, atol=1e-12)


def test_proj_psd_special_cases():
    rng = np.random.default_rng(3)
    Q = random_orthogonal(5, rng)
    Spos = (Q * rng.uniform(0.1, 2, 5)) @ Q.T
    Sneg = -Spos
    assert np.allclose(oracle.smat(oracle.proj_psd(oracle.svec(Spos))[0]), Spos, atol=1e-13)
    assert np.allclose(oracle.proj_psd(oracle.svec(Sneg))[0], 0.0, atol=1e-13)
    assert np.isclose(oracle.proj_psd(np.array([-3.0]))[0][0], 0.0)
    assert np.isclose(oracle.proj_psd(np.array([2.5]))[0][0], 2.5)
    # p = 2 in closed form: eigenvalues (a+c)/2 +- sqrt(((a-c)/2)^2 + b^2)
    a, bb, c = 0.3, 1.1, -0.7
    S = np.array([[a, bb], [bb, c]])
    r = math.hypot((a - c) / 2, bb)
    lp = (a + c) / 2 + r
    v = np.array([bb, lp - a]); v /= np.linalg.norm(v)
    assert np.allclose(oracle.smat(oracle.proj_psd(oracle.svec(S))[0]), lp * np.outer(v, v), atol=1e-14)


# --- Daleckii-Krein VJP ------------------------------------------------------

def _fd_proj(S, E, h):
    f = lambda t: oracle.smat(oracle.proj_psd(oracle.svec(S + t * E))[0])
    return (f(h) - f(-h)) / (2 * h)


def _dk_dir(S, E):
    _, U, lam = oracle.proj_psd(oracle.svec(S))
    return oracle.smat(oracle.psd_vjp_dk(U, lam, oracle.svec(E)))


@pytest.mark.parametrize("centers,delta", [(None, 1.0), ((-1.0, 1.0), 1e-4), ((-1.0, 1.0), 1e-10),
                                           ((0.5, 2.0), 1e-10)])
def test_dk_matches_finite_differences_on_clustered_spectra(centers, delta):
    # App. C sampler (two eigenvalue clusters), p = 40; the FD step never lets
    # an eigenvalue cross 0, so Pi is smooth along the segment.
    rng = np.random.default_rng(5)
    S, lam = appc_matrix(40, delta, rng, centers)
    E = _sym(rng, 40)
    h = 1e-6 if centers is not None else 1e-5
    fd = _fd_proj(S, E, h)
    # Pi is linear along directions inside one cluster only; compare the
    # self-adjoint directional derivative <G, D(E)> for random G as well.
    dk = _dk_dir(S, E)
    assert np.linalg.norm(dk - fd) <= 1e-7 * max(1.0, np.linalg.norm(fd))


def test_dk_exactly_repeated_eigenvalues_finite_and_correct():
    rng = np.random.default_rng(9)
    Q = random_orthogonal(8, rng)
    lam = np.array([-1, -1, -1, 2, 2, 2, 2, 0.5])
    S = (Q * lam) @ Q.T
    S = 0.5 * (S + S.T)
    E = _sym(rng, 8)
    dk = _dk_dir(S, E)
    assert np.all(np.isfinite(dk))
    assert np.linalg.norm(dk - _fd_proj(S, E, 1e-6)) < 1e-8 * np.linalg.norm(dk)
    # the eigendecomposition rule of eq:psd-cotangent is not finite here
    _, U, lam_c = oracle.proj_psd(oracle.svec(S))
    lam_c[1] = lam_c[0]  # force the exact tie that the theory has
    with np.errstate(all="ignore"):
        naive = oracle.psd_vjp_naive(U, lam_c, oracle.svec(E))
    assert not np.all(np.isfinite(naive))


def test_dk_self_adjoint_and_special_cases():
    rng = np.random.default_rng(13)
    S = _sym(rng, 9)
    _, U, lam = oracle.proj_psd(oracle.svec(S))
    G, E = oracle.svec(_sym(rng, 9)), oracle.svec(_sym(rng, 9))
    lhs = oracle.psd_vjp_dk(U, lam, G) @ E
    rhs = G @ oracle.psd_vjp_dk(U, lam, E)
    assert abs(lhs - rhs) < 1e-12
    # all eigenvalues positive -> identity; all negative -> zero
    Q = random_orthogonal(6, rng)
    lp = rng.uniform(0.5, 2.0, 6)
    for sgn, expect in ((1.0, "id"), (-1.0, "zero")):
        _, U2, l2 = oracle.proj_psd(oracle.svec((Q * (sgn * lp)) @ Q.T))
        G6 = oracle.svec(_sym(rng, 6))
        out = oracle.psd_vjp_dk(U2, l2, G6)
        assert np.allclose(out, G6 if expect == "id" else 0.0, atol=1e-12)
    # diagonal S: Sbar = L o Gbar with L the divided differences of max(.,0)
    d = np.array([-2.0, -0.5, 1.0, 3.0])
    Gm = _sym(rng, 4)
    _, U3, l3 = oracle.proj_psd(oracle.svec(np.diag(d)))
    out = oracle.smat(oracle.psd_vjp_dk(U3, l3, oracle.svec(Gm)))
    Lm = np.array([[1.0 if (a > 0 and b > 0) else (0.0 if (a <= 0 and b <= 0) else max(a, b) / (abs(a) + abs(b)))
                    for b in d] for a in d])
    assert np.allclose(out, Lm * Gm, atol=1e-13)


# --- SOC --------------------------------------------------------------------

def test_soc_projection_moreau_and_cases():
    rng = np.random.default_rng(21)
    for d in (2, 3, 7, 10):
        for _ in range(20):
            v = rng.standard_normal(d) * 2
            p, pm = oracle.proj_soc(v), oracle.proj_soc(-v)
            assert np.allclose(v, p - pm, atol=1e-13)          # SOC is self-dual
            assert abs(p @ (p - v)) < 1e-12
            assert np.linalg.norm(p[1:]) <= p[0] + 1e-12
    v = np.array([3.0, 1.0, 2.0])
    assert np.allclose(oracle.proj_soc(v), v)
    assert np.allclose(oracle.proj_soc(np.array([-3.0, 1.0, 2.0])), 0.0)


def test_soc_vjp_matches_fd():
    rng = np.random.default_rng(22)
    for d in (3, 6, 10):
        for _ in range(10):
            v = rng.standard_normal(d)
            g = rng.standard_normal(d)
            e = rng.standard_normal(d)
            h = 1e-7
            fd = (oracle.proj_soc(v + h * e) - oracle.proj_soc(v - h * e)) / (2 * h)
            assert abs(oracle.proj_soc_vjp(v, g) @ e - g @ fd) < 1e-6 * max(1.0, np.linalg.norm(g))


# --- rectification ----------------------------------------------------------

def test_rectify_block_means_and_adjoint():
    cones = [synth.Cone("zero", 2), synth.Cone("nonneg", 3), synth.Cone("soc", 3), synth.Cone("psd", 2)]
    rho = np.arange(1.0, 12.0)
    r = oracle.rectify(rho, cones)
    assert np.allclose(r[:5], rho[:5])
    assert np.allclose(r[5:8], 7.0) and np.allclose(r[8:11], 10.0)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(11), rng.standard_normal(11)
    assert np.isclose(oracle.rectify(a, cones) @ b, a @ oracle.rectify_adjoint(b, cones))


def test_lowner_ties_at_zero_take_the_nonpositive_side():
    """Reading R8: at an exact tie on the kink of max(., 0) the Loewner entry
    is the limit of the divided differences from the non-positive side
    (f'(0) = 0), a valid element of the generalized Jacobian; entries pairing
    0 with a positive eigenvalue stay ordinary divided differences.  The
    limits are taken on the oracle's divided differences of distinct values
    (pinned separately by finite differences), not on its tie branch."""
    L = oracle.lowner_matrix(np.array([0.0, 0.0, 2.0, -1.0, 0.0]))
    for eps in (1e-3, 1e-6, 1e-9):
        near = oracle.lowner_matrix(np.array([-eps, -2 * eps, 2.0, -1.0, -3 * eps]))
        assert np.allclose(L[[0, 1, 4]][:, [0, 1, 4]], near[[0, 1, 4]][:, [0, 1, 4]], atol=0.0)
    assert L[0, 0] == 0.0 and L[0, 1] == 0.0 and L[4, 4] == 0.0
    assert L[0, 2] == L[2, 0] == 1.0          # (f(2) - f(0)) / (2 - 0)
    assert L[0, 3] == L[3, 0] == 0.0          # (f(-1) - f(0)) / (-1 - 0)
    assert L[2, 2] == 1.0 and L[3, 3] == 0.0
