"""The five benchmark workloads as seeded synthetic batches, plus the
hyperparameter sequences and the App. B / App. C samplers.

Seeds: workload k >= 2 uses SeedSequence(k).spawn(B), instance i drawn from
child i; the single max-cut instance uses default_rng(0).  Data are generated
in float64; callers round them with ConicInstance.astype for float32 runs.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np
import scipy.sparse as sp

from .conic import PSD, SOC, ZERO, Cone, ConicInstance
from .graphs import erdos_renyi, random_circulant
from .problems import covsteer_sdp, huber_socp, lovasz_theta_sdp, maxcut_sdp


def _children(seed: int, B: int) -> List[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(B)]


def c1_instance() -> ConicInstance:
    """Single max-cut SDP on G(20, 0.3), unit weights, seed 0."""
    rng = np.random.default_rng(0)
    return maxcut_sdp(20, erdos_renyi(20, 0.3, rng))


def c2_batch(B: int = 64, p_lo: int = 30, p_hi: int = 100, seed: int = 2) -> List[ConicInstance]:
    """Max-cut SDPs, order p ~ U{p_lo..p_hi}, edge prob ~ U(0.1, 0.5)."""
    out = []
    for rng in _children(seed, B):
        p = int(rng.integers(p_lo, p_hi + 1))
        pe = float(rng.uniform(0.1, 0.5))
        out.append(maxcut_sdp(p, erdos_renyi(p, pe, rng)))
    return out


def c3_batch(B: int = 32, n_lo: int = 64, n_hi: int = 200, seed: int = 3) -> List[ConicInstance]:
    """Lovasz theta SDPs on random circulant (vertex-transitive) graphs."""
    out = []
    for rng in _children(seed, B):
        n = int(rng.integers(n_lo, n_hi + 1))
        S, edges = random_circulant(n, rng)
        inst = lovasz_theta_sdp(n, edges)
        inst.meta["conn"] = S
        out.append(inst)
    return out


def c4_batch(B: int = 256, seed: int = 4, n_obs: int = 2000, n_coef: int = 500,
             n_soc: int = 200) -> List[ConicInstance]:
    return [huber_socp(rng, n_obs=n_obs, n_coef=n_coef, n_soc=n_soc) for rng in _children(seed, B)]


def c5_batch(B: int = 128, seed: int = 5, nx_choices=(4, 6, 8, 10, 12),
             T_lo: int = 30, T_hi: int = 100) -> List[ConicInstance]:
    out = []
    for rng in _children(seed, B):
        nx = int(rng.choice(nx_choices))
        T = int(rng.integers(T_lo, T_hi + 1))
        out.append(covsteer_sdp(rng, nx, T))
    return out


def default_rho(inst: ConicInstance, K: int, rho0: float = 0.1, eq_scale: float = 1e3) -> np.ndarray:
    """[K, m] penalties: zero-cone rows rho0*eq_scale, all others rho0
    (Table 2 initial values (100, 0.1, 0.1, 0.1); fixed 1e3 equality scaling)."""
    r = np.full(inst.m, rho0)
    row = 0
    for c in inst.cones:
        if c.kind == ZERO:
            r[row:row + c.rows] = rho0 * eq_scale
        row += c.rows
    return np.tile(r, (K, 1))


def perturbed_hyper(inst: ConicInstance, K: int, rng: np.random.Generator,
                    rho0: float = 0.1, eq_scale: float = 1e3, spread: float = 0.5,
                    alpha_range=(1.4, 1.8)) -> Tuple[np.ndarray, np.ndarray]:
    """Per-(k, row) log-uniform perturbation of the default penalties and
    alpha^k ~ U(alpha_range): a stand-in for a policy's per-iteration output."""
    base = default_rho(inst, K, rho0, eq_scale)
    rho = base * np.exp(rng.uniform(-spread, spread, size=base.shape))
    alpha = rng.uniform(alpha_range[0], alpha_range[1], size=K)
    return rho, alpha


def appb_instance(n: int, rng: np.random.Generator, density: float = 0.01):
    """App. B sampler: diagonal P ~ U(0, 10); A (m = n/2) with `density` of
    entries N(0, 1); rho ~ U(0, 1); b ~ N(0, 1); target x* ~ N(0, 1)."""
    m = n // 2
    P = sp.diags(rng.uniform(0.0, 10.0, size=n)).tocsr()
    A = sp.random(m, n, density=density, format="csr", random_state=rng,
                  data_rvs=rng.standard_normal)
    rho = rng.uniform(0.0, 1.0, size=m)
    b = rng.standard_normal(m)
    xstar = rng.standard_normal(n)
    return P, A, rho, b, xstar


def random_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))


def appc_matrix(n: int, delta: float, rng: np.random.Generator,
                centers: Optional[Tuple[float, float]] = None) -> Tuple[np.ndarray, np.ndarray]:
    """App. C sampler: half of the eigenvalues near c1, half near c2
    (default -delta/2, +delta/2), spread sigma = 1e-3 delta, S = Q diag(l) Q'."""
    assert n % 2 == 0
    c1, c2 = centers if centers is not None else (-delta / 2, delta / 2)
    sig = delta * 1e-3
    lam = np.concatenate([c1 + rng.uniform(-sig, sig, n // 2),
                          c2 + rng.uniform(-sig, sig, n // 2)])
    Q = random_orthogonal(n, rng)
    S = (Q * lam) @ Q.T
    return 0.5 * (S + S.T), lam
