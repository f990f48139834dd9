"""The backward's per-step tap (cosmo_plan_set_tap) against the float64
oracle: at every unrolled step, the projection's input v^k and the cotangent
the reverse pass delivers to the projection's output (the cotangent of s+
net of the dual update's share), on every row."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import ensure_lib, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _oracle_taps(inst, rho, alpha, z0):
    """Per step k: (v^k, cotangent of s^{k+1} = Pi(v^k)) of the residual loss."""
    tape, (x, s, y) = oracle.unroll_forward(inst, rho, alpha, *z0)
    gx, gs, gy = oracle.residual_loss_grad(inst, x, s, y)
    out = [None] * len(tape)
    for k in range(len(tape) - 1, -1, -1):
        st = tape[k]
        out[k] = (st["v"], gs - st["rho_hat"] * gy)
        gx, gs, gy, _, _ = oracle.step_backward(inst, st, gx, gs, gy)
    return out


def _check(insts, K, rng, tol):
    from paper_2606_13825_amd import CosmoBatch
    rhos, alphas = zip(*(synth.perturbed_hyper(inst, K, rng) for inst in insts))
    z0 = [[rng.standard_normal(inst.n) for inst in insts], [rng.standard_normal(inst.m) for inst in insts],
          [rng.standard_normal(inst.m) for inst in insts]]
    batch = CosmoBatch(insts, K=K, dtype=torch.float64, device=DEV, cg_tol=1e-13, cg_max_iter=2000)
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(DEV)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(DEV)
    zt = [torch.from_numpy(np.concatenate(v)).to(DEV) for v in z0]
    fw = batch.forward(rho, alpha, *zt)
    _, g = batch.residual_loss(fw.x, fw.s, fw.y)
    tap = torch.zeros((K, 2, batch.m_tot), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        batch.set_tap(tap[:, :1])
    batch.set_tap(tap)
    batch.backward(rho, alpha, fw.tape, *g)
    batch.set_tap(None)
    bw_plain = batch.backward(rho, alpha, fw.tape, *g)   # recorded again without the tap
    torch.cuda.synchronize()
    assert torch.isfinite(bw_plain.grho).all()
    tp = tap.cpu().numpy()
    worst = 0.0
    for i, inst in enumerate(insts):
        ref = _oracle_taps(inst, rhos[i], alphas[i], [z[i] for z in z0])
        sl = slice(batch.m_off[i], batch.m_off[i + 1])
        scale_v = max(np.linalg.norm(r[0]) for r in ref)
        scale_g = max(np.linalg.norm(r[1]) for r in ref)
        for k in range(K):
            v_gpu, g_gpu = tp[k, 0, sl], tp[k, 1, sl]
            ev = np.linalg.norm(v_gpu - ref[k][0]) / max(np.linalg.norm(ref[k][0]), 1e-3 * scale_v)
            eg = np.linalg.norm(g_gpu - ref[k][1]) / max(np.linalg.norm(ref[k][1]), 1e-3 * scale_g)
            assert ev <= tol and eg <= tol, f"inst {i} step {k}: v error {ev:.2e}, cotangent error {eg:.2e}"
            worst = max(worst, ev, eg)
    say(f"  worst tap error {worst:.2e}")


def test_tap_mixed_cones_fp64():
    ensure_lib()
    rng = np.random.default_rng(41)
    insts = [synth.random_mixed(rng, n=8, soc_dims=(3, 4), psd_orders=(3, 2)),
             synth.random_mixed(rng, n=12, n_zero=0, soc_dims=(5,), psd_orders=(4,)),
             synth.random_mixed(rng, n=6, n_nonneg=0, soc_dims=(), psd_orders=(5, 1))]
    say("tap: mixed cones fp64 K=8")
    _check(insts, 8, rng, 1e-9)


def test_tap_double_integrator_fp64():
    """The covariance-steering instance of the trajectory study (one PSD block
    of order 44), from a random iterate."""
    ensure_lib()
    rng = np.random.default_rng(42)
    inst = synth.double_integrator_cs(rng)
    say(f"tap: double integrator n={inst.n} m={inst.m} fp64 K=20")
    _check([inst], 20, rng, 1e-8)
