"""GPU parity of the paper's comparison backward rules of the PSD projection
(eigendecomposition rule, Tikhonov shift, Newton-Schulz) against the float64
oracle on the same inputs, and the behaviour on exact eigenvalue ties that
distinguishes them from the Daleckii-Krein rule."""
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


def _spaced(rng, p):
    """Eigenvalues on a grid of +-[0.5, 2.5] (spacing >= 2/p, both signs),
    random eigenvectors: the eigendecomposition rule is well conditioned."""
    lam = np.linspace(0.5, 2.5, p) * np.where(rng.permutation(p) % 2 == 0, 1.0, -1.0)
    Q = random_orthogonal(p, rng)
    S = (Q * lam) @ Q.T
    return 0.5 * (S + S.T)


def _decompose(mats, dtype):
    from paper_2606_13825_amd import psd_proj
    orders = [m.shape[0] for m in mats]
    x = torch.from_numpy(np.concatenate([oracle.svec(m) for m in mats]).astype(dtype)).to(DEV)
    _, lam, U = psd_proj(x, orders, max_sweeps=60)
    return lam, U, orders


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-4), (np.float64, 1e-10)])
@pytest.mark.parametrize("rule,eps", [("naive", 0.0), ("tikhonov", 1e-3), ("tikhonov", 0.7)])
def test_eigendecomposition_rules_match_oracle(dtype, tol, rule, eps):
    ensure_lib()
    from paper_2606_13825_amd import psd_proj_vjp_rule
    rng = np.random.default_rng(11)
    mats = [_spaced(rng, p).astype(dtype).astype(np.float64) for p in (2, 3, 16, 17, 40, 64, 100)]
    G = [_sym(rng, m.shape[0]) for m in mats]
    g = np.concatenate([oracle.svec(x) for x in G]).astype(dtype)
    say(f"psd rule {rule} eps={eps} dtype={np.dtype(dtype).name}")
    lam, U, orders = _decompose(mats, dtype)
    gin = psd_proj_vjp_rule(lam, U, torch.from_numpy(g).to(DEV), orders, rule=rule, eps=eps)
    torch.cuda.synchronize()
    gin = gin.double().cpu().numpy()
    off = 0
    for S, Gm in zip(mats, G):
        p = S.shape[0]
        nr = p * (p + 1) // 2
        gv = oracle.svec(Gm).astype(dtype).astype(np.float64)
        if rule == "naive":
            _, Ur, lr = oracle.proj_psd(oracle.svec(S))
            ref = oracle.psd_vjp_naive(Ur, lr, gv)
        else:
            ref = oracle.psd_vjp_tikhonov(oracle.svec(S), eps, gv)
        e = rel_err(gin[off:off + nr], ref, 1e-6 * np.linalg.norm(gv))
        assert e <= tol, (rule, p, e)
        off += nr


def test_dk_rule_entry_equals_psd_proj_vjp():
    ensure_lib()
    from paper_2606_13825_amd import psd_proj_vjp, psd_proj_vjp_rule
    rng = np.random.default_rng(12)
    mats = [_sym(rng, p) for p in (5, 40, 100)]
    lam, U, orders = _decompose(mats, np.float32)
    g = torch.from_numpy(np.concatenate([oracle.svec(_sym(rng, p)) for p in orders]).astype(np.float32)).to(DEV)
    a = psd_proj_vjp(lam, U, g, orders)
    b = psd_proj_vjp_rule(lam, U, g, orders, rule="dk", eps=5.0)   # eps is ignored by the DK rule
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_exact_ties_break_the_eigendecomposition_rule_only():
    # diagonal blocks: the eigensolver returns the diagonal exactly, so ties
    # are exact.  eq:psd-cotangent is not finite there; DK and Newton-Schulz are.
    ensure_lib()
    from paper_2606_13825_amd import NewtonSchulzProj, psd_proj_vjp_rule
    d = np.array([2.0, 2.0, -1.0, 0.5, -1.0, 3.0])
    S = np.diag(d)
    rng = np.random.default_rng(13)
    Gm = _sym(rng, 6)
    gv = oracle.svec(Gm)
    lam, U, orders = _decompose([S], np.float64)
    g = torch.from_numpy(gv).to(DEV)
    naive = psd_proj_vjp_rule(lam, U, g, orders, rule="naive").cpu().numpy()
    dk = psd_proj_vjp_rule(lam, U, g, orders, rule="dk").cpu().numpy()
    ns = NewtonSchulzProj(orders, 40, torch.float64, DEV)
    ns.forward(torch.from_numpy(oracle.svec(S)).to(DEV))
    nsg = ns.vjp(g).cpu().numpy()
    assert not np.all(np.isfinite(naive))
    assert np.all(np.isfinite(dk)) and np.all(np.isfinite(nsg))
    _, Ur, lr = oracle.proj_psd(oracle.svec(S))
    ref = oracle.psd_vjp_dk(Ur, lr, gv)
    assert rel_err(dk, ref) <= 1e-12
    assert rel_err(nsg, ref) <= 1e-10


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-4), (np.float64, 1e-10)])
def test_newton_schulz_matches_oracle(dtype, tol):
    ensure_lib()
    from paper_2606_13825_amd import NewtonSchulzProj
    rng = np.random.default_rng(14)
    mats = [_spaced(rng, p) for p in (1, 2, 3, 16, 17, 33, 64, 100)]
    mats.append(appc_matrix(40, 1e-5, rng)[0])               # App. C sampler, gap 1e-5
    mats.append(_spaced(rng, 250))                            # beyond the eigensolver's orders
    mats = [m.astype(dtype).astype(np.float64) for m in mats]
    orders = [m.shape[0] for m in mats]
    K = 24
    x = np.concatenate([oracle.svec(m) for m in mats])
    G = [_sym(rng, p) for p in orders]
    g = np.concatenate([oracle.svec(m) for m in G]).astype(dtype)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    say(f"newton-schulz parity dtype={np.dtype(dtype).name} K={K} orders={orders}")
    ns = NewtonSchulzProj(orders, K, tdt, DEV)
    out = ns.forward(torch.from_numpy(x.astype(dtype)).to(DEV))
    gin = ns.vjp(torch.from_numpy(g).to(DEV))
    # the tape stays valid: a second reverse pass gives the same bits
    gin2 = ns.vjp(torch.from_numpy(g).to(DEV))
    torch.cuda.synchronize()
    assert torch.equal(gin, gin2)
    out = out.double().cpu().numpy()
    gin = gin.double().cpu().numpy()
    off = 0
    for S, Gm in zip(mats, G):
        p = S.shape[0]
        nr = p * (p + 1) // 2
        v = oracle.svec(S)
        ref_out, tape = oracle.ns_forward(v, K)
        gv = oracle.svec(Gm).astype(dtype).astype(np.float64)
        ref_g = oracle.ns_vjp(tape, gv)
        eo = rel_err(out[off:off + nr], ref_out, 1e-6 * np.linalg.norm(v))
        eg = rel_err(gin[off:off + nr], ref_g, 1e-6 * np.linalg.norm(gv))
        assert eo <= tol and eg <= tol, (p, eo, eg)
        off += nr


def test_newton_schulz_zero_steps_and_reuse_with_other_sizes():
    # K = 0 (Pi = S/2 + S^2 / (2 ||S||_F)) and a second object with other
    # orders and step count on the same stream.
    ensure_lib()
    from paper_2606_13825_amd import NewtonSchulzProj
    rng = np.random.default_rng(15)
    for orders, K in (([7, 31, 32], 0), ([5, 48], 3)):
        mats = [_sym(rng, p) for p in orders]
        x = np.concatenate([oracle.svec(m) for m in mats])
        g = np.concatenate([oracle.svec(_sym(rng, p)) for p in orders])
        ns = NewtonSchulzProj(orders, K, torch.float64, DEV)
        out = ns.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
        gin = ns.vjp(torch.from_numpy(g).to(DEV)).cpu().numpy()
        off = 0
        for p, S in zip(orders, mats):
            nr = p * (p + 1) // 2
            ro, tape = oracle.ns_forward(x[off:off + nr], K)
            rg = oracle.ns_vjp(tape, g[off:off + nr])
            assert rel_err(out[off:off + nr], ro) <= 1e-12
            assert rel_err(gin[off:off + nr], rg) <= 1e-11
            off += nr


def test_rule_errors_against_finite_differences_over_the_gap():
    """The appendix's accuracy experiment in float64: App. C matrices of order
    40 with two eigenvalue clusters at +-delta/2, delta from 1 to 1e-10; each
    rule's directional derivative <gin, E> against central differences of the
    float64 projection along E.  DK and Newton-Schulz stay accurate at every
    gap, the eigendecomposition rule stays finite on these (distinct)
    eigenvalues, Tikhonov with eps = 1e-3 is biased once eps exceeds the gap."""
    ensure_lib()
    from paper_2606_13825_amd import NewtonSchulzProj, psd_proj_vjp_rule
    rng = np.random.default_rng(16)
    n, K = 40, 30
    deltas = (1.0, 1e-2, 1e-4, 1e-6, 1e-8, 1e-10)
    mats = [appc_matrix(n, d, rng)[0] for d in deltas]
    G = [_sym(rng, n) for _ in deltas]
    E = [[_sym(rng, n) for _ in range(3)] for _ in deltas]
    orders = [n] * len(deltas)
    x = torch.from_numpy(np.concatenate([oracle.svec(m) for m in mats])).to(DEV)
    g = torch.from_numpy(np.concatenate([oracle.svec(m) for m in G])).to(DEV)
    lam, U, _ = _decompose(mats, np.float64)
    out = {r: psd_proj_vjp_rule(lam, U, g, orders, rule=r, eps=1e-3).cpu().numpy()
           for r in ("dk", "naive", "tikhonov")}
    ns = NewtonSchulzProj(orders, K, torch.float64, DEV)
    ns.forward(x)
    out["ns"] = ns.vjp(g).cpu().numpy()
    nr = n * (n + 1) // 2
    for b, (d, S, Gm) in enumerate(zip(deltas, mats, G)):
        h = 1e-4 * d                  # no eigenvalue reaches 0 along the segment
        errs = {r: 0.0 for r in out}
        for Em in E[b]:
            fd = (oracle.proj_psd(oracle.svec(S + h * Em))[0] - oracle.proj_psd(oracle.svec(S - h * Em))[0]) / (2 * h)
            ref = oracle.svec(Gm) @ fd
            for r, gin in out.items():
                errs[r] = max(errs[r], abs(gin[b * nr:(b + 1) * nr] @ oracle.svec(Em) - ref) / abs(ref))
        say(f"delta={d:.0e} " + " ".join(f"{r}={e:.2e}" for r, e in errs.items()))
        # the differences themselves carry ~1e-6 (truncation of the curvature
        # ~1/delta at step 1e-4 delta)
        assert errs["dk"] <= 1e-5 and errs["ns"] <= 1e-5, (d, errs)
        assert np.all(np.isfinite(out["naive"][b * nr:(b + 1) * nr]))
        if d <= 1e-4:
            assert errs["tikhonov"] >= 0.1, (d, errs)
        if d == 1.0:
            assert errs["tikhonov"] <= 1e-2, (d, errs)


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-4), (np.float64, 1e-10)])
def test_newton_schulz_many_blocks_large_product_tiles(dtype, tol):
    # enough 64 x 64 output tiles (>= 512) that the products run in the
    # 2 x 2-blocked form; orders 20..70 put partial tiles everywhere.  Every
    # 8th block is checked against the oracle, all blocks for finiteness.
    ensure_lib()
    from paper_2606_13825_amd import NewtonSchulzProj
    rng = np.random.default_rng(17)
    orders = [int(p) for p in rng.integers(20, 71, size=512)]
    K = 12
    mats = [_spaced(rng, p).astype(dtype).astype(np.float64) for p in orders]
    x = np.concatenate([oracle.svec(m) for m in mats])
    g = np.concatenate([oracle.svec(_sym(rng, p)) for p in orders]).astype(dtype)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    say(f"newton-schulz 512 blocks dtype={np.dtype(dtype).name} K={K}")
    ns = NewtonSchulzProj(orders, K, tdt, DEV)
    out = ns.forward(torch.from_numpy(x.astype(dtype)).to(DEV)).double().cpu().numpy()
    gin = ns.vjp(torch.from_numpy(g).to(DEV)).double().cpu().numpy()
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(gin))
    off = 0
    for b, p in enumerate(orders):
        nr = p * (p + 1) // 2
        if b % 8 == 0:
            v = x[off:off + nr]
            ro, tape = oracle.ns_forward(v, K)
            gv = g[off:off + nr].astype(np.float64)
            rg = oracle.ns_vjp(tape, gv)
            eo = rel_err(out[off:off + nr], ro, 1e-6 * np.linalg.norm(v))
            eg = rel_err(gin[off:off + nr], rg, 1e-6 * np.linalg.norm(gv))
            assert eo <= tol and eg <= tol, (b, p, eo, eg)
        off += nr
