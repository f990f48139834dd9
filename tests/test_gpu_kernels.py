"""Per-kernel parity on the GPU: PSD projection (Jacobi eigensolver + MFMA
reconstruction), Daleckii-Krein VJP (MFMA), SOC projection and VJP, against
the float64 oracle on the same inputs."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import ensure_lib, rel_err, say
from synth.workloads import appc_matrix, random_orthogonal

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _sym(rng, p):
    G = rng.standard_normal((p, p))
    return 0.5 * (G + G.T)


def _run_psd(mats, dtype):
    from paper_2606_13825_amd import psd_proj
    orders = [m.shape[0] for m in mats]
    x = np.concatenate([oracle.svec(m) for m in mats])
    xt = torch.from_numpy(x.astype(dtype)).to(DEV)
    out, lam, U = psd_proj(xt, orders, max_sweeps=60)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), lam, U, orders


@pytest.mark.parametrize("dtype,tol", [(np.float32, 2e-6), (np.float64, 1e-12)])
def test_psd_proj_sizes_and_tails(dtype, tol):
    ensure_lib()
    rng = np.random.default_rng(1)
    orders = [1, 2, 3, 5, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129]
    if dtype == np.float32:
        orders += [160, 199, 200]
    else:
        orders += [140]
    mats = [_sym(rng, p).astype(dtype).astype(np.float64) for p in orders]
    say(f"psd_proj parity dtype={np.dtype(dtype).name} orders={orders}")
    out, lam, U, _ = _run_psd(mats, dtype)
    off = 0
    for S in mats:
        p = S.shape[0]
        nr = p * (p + 1) // 2
        ref = oracle.proj_psd(oracle.svec(S))[0]
        e = rel_err(out[off:off + nr], ref, 1e-6 * np.linalg.norm(oracle.svec(S)))
        assert e <= tol * max(1.0, np.sqrt(p) / 4), (p, e)
        off += nr


def test_psd_proj_small_split_gap():
    """Blocks whose positive / non-positive split is narrow against their
    norm: an eigenvalue just below zero beside a small positive one, the rest
    spread to +-100 (the shape of a maxcut iterate block that once left
    1.3e-4 in the projection).  Float32 Jacobi cannot take such a pair's
    mixing angle below ~1e-3; the refinement's first-order rotation has to
    resolve it (or the block is solved again with converged sweeps)."""
    ensure_lib()
    rng = np.random.default_rng(5)
    mats = []
    for p, (neg, pos) in ((40, (-8.5e-4, 0.26)), (89, (-8.5e-4, 0.26)), (100, (-1e-2, 1e-2)),
                          (128, (-5e-3, 0.5)), (64, (-0.3, 0.3))):
        big = rng.uniform(1.0, 100.0, p - 2) * rng.choice([-1.0, 1.0], p - 2)
        lam = np.concatenate([[neg, pos], big])
        Q = random_orthogonal(p, rng)
        mats.append(((Q * lam) @ Q.T).astype(np.float32).astype(np.float64))
    mats = [0.5 * (m + m.T) for m in mats]
    say("psd_proj small split gaps, orders " + str([m.shape[0] for m in mats]))
    out, _, _, _ = _run_psd(mats, np.float32)
    off = 0
    for S in mats:
        p = S.shape[0]
        nr = p * (p + 1) // 2
        ref = oracle.proj_psd(oracle.svec(S))[0]
        e = rel_err(out[off:off + nr], ref, 1e-6 * np.linalg.norm(oracle.svec(S)))
        assert e <= 2e-6 * max(1.0, np.sqrt(p) / 4), (p, e)
        off += nr


@pytest.mark.parametrize("delta", [1.0, 1e-4, 1e-10])
def test_psd_proj_clustered_and_repeated_eigenvalues(delta):
    ensure_lib()
    rng = np.random.default_rng(2)
    mats = []
    for _ in range(4):
        S, _ = appc_matrix(40, delta, rng)
        mats.append(S.astype(np.float32).astype(np.float64))
    Q = random_orthogonal(12, rng)
    lam = np.array([-1, -1, -1, 2, 2, 2, 2, 0.5, 0.5, -3, 4, 4.0])
    mats.append(((Q * lam) @ Q.T).astype(np.float32).astype(np.float64))
    say(f"psd_proj clustered delta={delta}")
    out, _, _, _ = _run_psd([0.5 * (m + m.T) for m in mats], np.float32)
    off = 0
    for S in mats:
        S = 0.5 * (S + S.T)
        p = S.shape[0]
        nr = p * (p + 1) // 2
        ref = oracle.proj_psd(oracle.svec(S))[0]
        scale = np.linalg.norm(oracle.svec(S))
        assert np.linalg.norm(out[off:off + nr] - ref) <= 3e-6 * scale
        off += nr


def test_psd_eigenpairs_are_orthonormal_and_accurate():
    ensure_lib()
    rng = np.random.default_rng(3)
    mats = [_sym(rng, p).astype(np.float32).astype(np.float64) for p in (8, 40, 100)]
    _, lam, U, orders = _run_psd(mats, np.float32)
    lam = lam.double().cpu().numpy()
    U = U.double().cpu().numpy()
    lo = uo = 0
    for S, p in zip(mats, orders):
        Ub = U[uo:uo + p * p].reshape(p, p).T   # stored column-major
        lb = lam[lo:lo + p]
        assert np.linalg.norm(Ub.T @ Ub - np.eye(p)) <= 2e-5 * p
        ref = np.sort(np.linalg.eigvalsh(S))
        assert np.max(np.abs(np.sort(lb) - ref)) <= 2e-6 * max(1.0, np.abs(ref).max()) * np.sqrt(p)
        assert np.linalg.norm(S @ Ub - Ub * lb) <= 1e-5 * np.linalg.norm(S) * np.sqrt(p)
        lo += p
        uo += p * p


# Orders up to each dtype's maximum, across all four order classes: the
# largest (float32 200, float64 140) need the unpadded LDS layout of the
# VJP's first buffer.
@pytest.mark.parametrize("dtype,tol,orders", [
    (np.float32, 3e-5, (3, 16, 17, 40, 64, 100)),
    (np.float32, 3e-5, (129, 160, 199, 200)),
    (np.float64, 1e-11, (3, 16, 17, 40, 64, 100, 129, 140)),
])
def test_dk_vjp_matches_oracle(dtype, tol, orders):
    ensure_lib()
    from paper_2606_13825_amd import psd_proj_vjp
    rng = np.random.default_rng(4)
    mats = []
    for p in orders:
        mats.append(_sym(rng, p).astype(dtype).astype(np.float64))
    S2, _ = appc_matrix(40, 1e-8, rng, centers=(-1.0, 1.0))
    mats.append(S2.astype(dtype).astype(np.float64))
    say(f"dk vjp parity dtype={np.dtype(dtype).name}")
    _, lam, U, orders = _run_psd(mats, dtype)
    G = [_sym(rng, m.shape[0]) for m in mats]
    g = np.concatenate([oracle.svec(x) for x in G]).astype(dtype)
    gin = psd_proj_vjp(lam, U, torch.from_numpy(g).to(DEV), orders)
    torch.cuda.synchronize()
    gin = gin.double().cpu().numpy()
    off = 0
    errs = []
    for S, Gm in zip(mats, G):
        p = S.shape[0]
        nr = p * (p + 1) // 2
        _, Ur, lr = oracle.proj_psd(oracle.svec(S))
        ref = oracle.psd_vjp_dk(Ur, lr, oracle.svec(Gm).astype(dtype).astype(np.float64))
        e = rel_err(gin[off:off + nr], ref, 1e-6 * np.linalg.norm(oracle.svec(Gm)))
        errs.append((p, e))
        off += nr
    say("  rel err per order: " + ", ".join(f"{p}: {e:.1e}" for p, e in errs))
    for p, e in errs:
        assert e <= tol, (p, e)


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-6), (np.float64, 1e-13)])
def test_dk_vjp_ties_at_zero_match_oracle(dtype, tol):
    """Diagonal blocks with exactly repeated zero eigenvalues: the GPU's
    Loewner weights at ties on the kink (vjp_weight) take the same
    convention as the oracle's (f'(0) = 0, reading R8), so the VJPs agree."""
    ensure_lib()
    from paper_2606_13825_amd import psd_proj_vjp
    rng = np.random.default_rng(8)
    mats = [np.diag([0.0, 0.0, 2.0, -1.0, 0.0, 0.5]), np.diag([0.0] * 4 + [1.0] * 3),
            np.diag(np.r_[np.zeros(20), rng.uniform(0.5, 2.0, 20), -rng.uniform(0.5, 2.0, 20)])]
    _, lam, U, orders = _run_psd(mats, dtype)
    lam_h = lam.double().cpu().numpy()
    assert np.sum(lam_h == 0.0) == 3 + 4 + 20     # the zeros come out exactly
    G = [_sym(rng, m.shape[0]) for m in mats]
    g = np.concatenate([oracle.svec(x) for x in G]).astype(dtype)
    gin = psd_proj_vjp(lam, U, torch.from_numpy(g).to(DEV), orders)
    torch.cuda.synchronize()
    gin = gin.double().cpu().numpy()
    off = 0
    for S, Gm in zip(mats, G):
        p = S.shape[0]
        nr = p * (p + 1) // 2
        ref = oracle.psd_vjp_dk(np.eye(p), np.diag(S).copy(), oracle.svec(Gm).astype(dtype).astype(np.float64))
        assert rel_err(gin[off:off + nr], ref, 1e-6) <= tol, p
        off += nr


def test_soc_projection_and_vjp():
    ensure_lib()
    from paper_2606_13825_amd import socp_proj, socp_proj_vjp
    rng = np.random.default_rng(5)
    dims = [1, 2, 3, 4, 7, 10, 33]
    vs, gs = [], []
    for d in dims:
        for case in range(3):
            v = rng.standard_normal(d)
            if case == 0 and d > 1:
                v[0] = np.linalg.norm(v[1:]) * 1.5       # inside the cone
            elif case == 1 and d > 1:
                v[0] = -np.linalg.norm(v[1:]) * 1.5      # inside the polar cone
            vs.append(v)
            gs.append(rng.standard_normal(d))
    alld = [len(v) for v in vs]
    for dtype, tol in ((np.float32, 2e-6), (np.float64, 1e-13)):
        x = torch.from_numpy(np.concatenate(vs).astype(dtype)).to(DEV)
        g = torch.from_numpy(np.concatenate(gs).astype(dtype)).to(DEV)
        out = socp_proj(x, alld).double().cpu().numpy()
        gin = socp_proj_vjp(x, g, alld).double().cpu().numpy()
        off = 0
        for v, gg in zip(vs, gs):
            d = len(v)
            v32 = v.astype(dtype).astype(np.float64)
            g32 = gg.astype(dtype).astype(np.float64)
            assert rel_err(out[off:off + d], oracle.proj_soc(v32), 1e-6) <= tol
            assert rel_err(gin[off:off + d], oracle.proj_soc_vjp(v32, g32), 1e-6) <= tol * 10
            off += d
