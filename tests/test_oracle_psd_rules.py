"""Pins of the oracle's comparison backward rules of the PSD projection
(Tikhonov shift, Newton-Schulz sign iteration) against finite differences,
closed forms and the limits the mathematics fixes (CPU only)."""
import numpy as np
import pytest

import oracle
from synth.workloads import appc_matrix, random_orthogonal


def _sym(rng, p):
    G = rng.standard_normal((p, p))
    return 0.5 * (G + G.T)


def _separated(rng, p, lo=0.5, hi=2.0):
    """Symmetric matrix with eigenvalues in +-[lo, hi], both signs present."""
    Q = random_orthogonal(p, rng)
    lam = rng.uniform(lo, hi, p) * np.where(np.arange(p) % 2 == 0, 1.0, -1.0)
    S = (Q * lam) @ Q.T
    return 0.5 * (S + S.T)


@pytest.mark.parametrize("p", [2, 7, 16, 40])
def test_ns_forward_converges_to_eigen_projection(p):
    # eq:newton-schulz converges to sign(S) once ||S_k||_2 < 1; S_0 = S/||S||_F
    # guarantees it, so with enough steps (S + sign(S) S)/2 is eq:psd-proj.
    rng = np.random.default_rng(p)
    v = oracle.svec(_separated(rng, p))
    out, _ = oracle.ns_forward(v, 60)
    ref = oracle.proj_psd(v)[0]
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)


def test_ns_zero_steps_closed_form():
    # K = 0: Pi(S) = S/2 + S^2 / (2 ||S||_F); its derivative along E is
    # E/2 + (E S + S E) / (2c) - S^2 <S, E> / (2 c^3).
    rng = np.random.default_rng(1)
    S, E, G = _sym(rng, 6), _sym(rng, 6), _sym(rng, 6)
    c = np.linalg.norm(S)
    D = 0.5 * E + (E @ S + S @ E) / (2 * c) - S @ S * np.sum(S * E) / (2 * c ** 3)
    vjp = oracle.psd_vjp_ns(oracle.svec(S), 0, oracle.svec(G))
    assert abs(vjp @ oracle.svec(E) - np.sum(G * D)) <= 1e-13 * max(1.0, abs(np.sum(G * D)))
    out, _ = oracle.ns_forward(oracle.svec(S), 0)
    assert np.allclose(oracle.smat(out), 0.5 * S + S @ S / (2 * c), atol=1e-14)


@pytest.mark.parametrize("K", [1, 3, 8, 25])
def test_ns_vjp_matches_finite_differences(K):
    # reverse mode of the unrolled iteration against central differences of
    # the forward map itself (same K), on a generic symmetric matrix.
    rng = np.random.default_rng(10 + K)
    p = 9
    v = oracle.svec(_sym(rng, p))
    g = oracle.svec(_sym(rng, p))
    for _ in range(3):
        e = oracle.svec(_sym(rng, p))
        f = lambda t: oracle.ns_forward(v + t * e, K)[0] @ g
        h = 1e-5
        fd = (f(h) - f(-h)) / (2 * h)
        an = oracle.psd_vjp_ns(v, K, g) @ e
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)), (K, fd, an)


def test_ns_vjp_converges_to_dk():
    # where the spectrum stays away from 0 the converged sign iteration is
    # Pi itself on a neighbourhood, so its derivative is the DK derivative.
    rng = np.random.default_rng(3)
    for p in (5, 20):
        v = oracle.svec(_separated(rng, p))
        g = oracle.svec(_sym(rng, p))
        _, U, lam = oracle.proj_psd(v)
        dk = oracle.psd_vjp_dk(U, lam, g)
        ns = oracle.psd_vjp_ns(v, 60, g)
        assert np.linalg.norm(ns - dk) <= 1e-11 * np.linalg.norm(dk)


def test_tikhonov_is_the_derivative_of_the_shifted_projection():
    # with distinct eigenvalues eq:psd-cotangent equals the DK rule, so the
    # Tikhonov rule is the derivative of S -> Pi(S + eps I): compare with
    # central differences of that map.
    rng = np.random.default_rng(4)
    p, eps = 10, 1e-2
    S = _separated(rng, p)
    v, g = oracle.svec(S), oracle.svec(_sym(rng, p))
    I = oracle.svec(np.eye(p))
    tik = oracle.psd_vjp_tikhonov(v, eps, g)
    for _ in range(3):
        e = oracle.svec(_sym(rng, p))
        f = lambda t: oracle.proj_psd(v + eps * I + t * e)[0] @ g
        h = 1e-6
        fd = (f(h) - f(-h)) / (2 * h)
        assert abs(tik @ e - fd) <= 1e-7 * max(1.0, abs(fd))
    # eps = 0 reduces to the eigendecomposition rule at S
    _, U, lam = oracle.proj_psd(v)
    assert np.allclose(oracle.psd_vjp_tikhonov(v, 0.0, g), oracle.psd_vjp_naive(U, lam, g), atol=1e-12)


def test_tikhonov_bias_when_shift_exceeds_gap():
    # App. C sampler at gap delta = 1e-6 with eps = 1e-3 >> delta: the shift
    # moves the negative cluster across 0, so the rule is the derivative of a
    # different map; the DK rule at S is the true derivative.
    rng = np.random.default_rng(6)
    S, _ = appc_matrix(20, 1e-6, rng)
    v, g = oracle.svec(S), oracle.svec(_sym(rng, 20))
    _, U, lam = oracle.proj_psd(v)
    dk = oracle.psd_vjp_dk(U, lam, g)
    tik = oracle.psd_vjp_tikhonov(v, 1e-3, g)
    assert np.linalg.norm(tik - dk) > 0.1 * np.linalg.norm(dk)


def test_ns_finite_and_naive_not_on_exact_ties():
    # a diagonal matrix with a repeated eigenvalue: eigh returns the exact
    # tie, eq:psd-cotangent is not finite there, Newton-Schulz and DK are.
    d = np.array([2.0, 2.0, -1.0, 0.5, -1.0])
    v = oracle.svec(np.diag(d))
    rng = np.random.default_rng(8)
    g = oracle.svec(_sym(rng, 5))
    _, U, lam = oracle.proj_psd(v)
    with np.errstate(all="ignore"):
        assert not np.all(np.isfinite(oracle.psd_vjp_naive(U, lam, g)))
        assert not np.all(np.isfinite(oracle.psd_vjp_tikhonov(v, 1e-6, g)))
    ns = oracle.psd_vjp_ns(v, 40, g)
    dk = oracle.psd_vjp_dk(U, lam, g)
    assert np.all(np.isfinite(ns))
    assert np.linalg.norm(ns - dk) <= 1e-10 * np.linalg.norm(dk)
