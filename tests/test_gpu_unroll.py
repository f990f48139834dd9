"""End-to-end parity of the batched unrolled COSMO on the GPU against the
float64 oracle: every iterate of the tape, the final-residual loss, and the
gradients w.r.t. (rho^k, alpha^k, x0, s0, y0)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import assert_blocks_close, assert_close, ensure_lib, floor_bars, floor_of, oracle_run, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _stack_hyper(insts, K, rng, perturb=True, dtype=np.float32):
    rhos, alphas = [], []
    for inst in insts:
        if perturb:
            r, a = synth.perturbed_hyper(inst, K, rng)
        else:
            r, a = synth.default_rho(inst, K), np.full(K, 1.6)
        rhos.append(r.astype(dtype))
        alphas.append(a.astype(dtype))
    return rhos, alphas


def _run(insts, K, dtype, rhos, alphas, z0=None, cg_tol=None, grad=True, **kw):
    from paper_2606_13825_amd import CosmoBatch
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    batch = CosmoBatch(insts, K=K, dtype=tdt, device=DEV, cg_tol=cg_tol, **kw)
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(DEV)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(DEV)
    args = [None, None, None]
    if z0 is not None:
        args = [torch.from_numpy(np.concatenate(v).astype(dtype)).to(DEV) for v in z0]
    stats = batch.new_stats()
    fw = batch.forward(rho, alpha, *args, stats=stats)
    loss, g = batch.residual_loss(fw.x, fw.s, fw.y)
    bw = batch.backward(rho, alpha, fw.tape, *g, stats=stats) if grad else None
    torch.cuda.synchronize()
    return batch, fw, loss, bw, batch.stats_dict(stats)


def _check(batch, fw, loss, bw, insts, rhos, alphas, tol_it, tol_g, every_k=False, z0=None, grad=True, cg_tol=0.0):
    for i, inst in enumerate(insts):
        zi = None if z0 is None else [z0[0][i], z0[1][i], z0[2][i]]
        r64, a64 = rhos[i].astype(np.float64), alphas[i].astype(np.float64)
        ref = oracle_run(inst, r64, a64, grad, *(zi if zi else (None, None, None)))
        fl = floor_of(inst)
        runs = []
        if batch.dtype == torch.float32:   # bars from the instance's float32 floor (gpu_common)
            tol_it_i, tol_g_i, (f_it, f_g) = floor_bars(inst, r64, a64, ref, tol_it, tol_g,
                                                        **(dict(zip(("x0", "s0", "y0"), zi)) if zi else {}),
                                                        with_grad=grad, cg_tol=cg_tol, runs=runs)
            say(f"  inst {i}: float32 floor {f_it:.1e} (iterates) {f_g:.1e} (gradients); "
                f"bars {tol_it_i:.1e} {tol_g_i:.1e}")
        else:
            tol_it_i, tol_g_i = tol_it, tol_g
        sl_n = slice(batch.n_off[i], batch.n_off[i + 1])
        sl_m = slice(batch.m_off[i], batch.m_off[i + 1])
        if every_k:
            # Every iterate against its own norm, floored at a tenth of the
            # largest norm the same array reaches over the K steps: early
            # iterates can be small, and float32 rounding of b - A x~ on
            # equality rows is amplified by rho_hat in y+ (about 7e-6 of the
            # first dual iterate of a max-cut step from that term alone).
            scale = {nm: max(np.linalg.norm(st[key]) for st in ref["tape"])
                     for nm, key in (("x", "xn"), ("s", "sn"), ("y", "yn"))}
            for k in range(1, batch.K + 1):
                x, s, y, _, _ = batch.tape_iterate(fw.tape, k)
                st = ref["tape"][k - 1]
                for nm, g_, r_ in (("x", x[sl_n], st["xn"]), ("s", s[sl_m], st["sn"]), ("y", y[sl_m], st["yn"])):
                    assert_close(g_.double().cpu().numpy(), r_, tol_it_i, max(fl, 0.1 * scale[nm]),
                                 f"inst {i} iterate {nm}^{k}")
        for nm, g_, r_ in (("x", fw.x[sl_n], ref["x"]), ("s", fw.s[sl_m], ref["s"]), ("y", fw.y[sl_m], ref["y"])):
            assert_close(g_.double().cpu().numpy(), r_, tol_it_i, fl, f"inst {i} final {nm}")
        for nm, g_, r_ in (("s", fw.s[sl_m], ref["s"]), ("y", fw.y[sl_m], ref["y"])):
            assert_blocks_close(g_.double().cpu().numpy(), r_, inst, tol_it, f"inst {i} final {nm}", floor=fl,
                                floor_runs=[run[1 if nm == "s" else 2] for run in runs])
        assert abs(float(loss[i]) - ref["loss"]) <= tol_g_i * max(abs(ref["loss"]), 1e-6), (i, float(loss[i]),
                                                                                           ref["loss"])
        if grad:
            assert_close(bw.grho[:, sl_m].double().cpu().numpy(), ref["grho"], tol_g_i, 0.0, f"inst {i} grad rho")
            assert_close(bw.galpha[:, i].double().cpu().numpy(), ref["galpha"], tol_g_i, 0.0, f"inst {i} grad alpha")
            for nm, g_, r_ in (("x0", bw.gx0[sl_n], ref["gx0"]), ("s0", bw.gs0[sl_m], ref["gs0"]),
                               ("y0", bw.gy0[sl_m], ref["gy0"])):
                assert_close(g_.double().cpu().numpy(), r_, tol_g_i, 1e-6 * max(1.0, np.linalg.norm(ref["grho"])),
                             f"inst {i} grad {nm}")


@pytest.mark.parametrize("dtype,tol_it,tol_g", [(np.float64, 1e-10, 1e-8), (np.float32, 1e-5, 1e-4)])
def test_mixed_cones_every_iterate_and_gradients(dtype, tol_it, tol_g):
    ensure_lib()
    rng = np.random.default_rng(10)
    insts = [synth.random_mixed(rng, n=8, soc_dims=(3, 4), psd_orders=(3, 2)),
             synth.random_mixed(rng, n=12, n_zero=0, soc_dims=(5,), psd_orders=(4,)),
             synth.random_mixed(rng, n=6, n_nonneg=0, soc_dims=(), psd_orders=(5, 1))]
    insts = [x.astype(dtype) for x in insts]
    K = 8
    rhos, alphas = _stack_hyper(insts, K, rng, dtype=dtype)
    z0 = [[(0.3 * rng.standard_normal(d)).astype(dtype) for d in (x.n for x in insts)],
          [(0.3 * rng.standard_normal(d)).astype(dtype) for d in (x.m for x in insts)],
          [(0.3 * rng.standard_normal(d)).astype(dtype) for d in (x.m for x in insts)]]
    z0d = [[v.astype(np.float64) for v in grp] for grp in z0]
    say(f"mixed cones dtype={np.dtype(dtype).name} K={K}")
    cg = 1e-13 if dtype == np.float64 else 1e-7
    batch, fw, loss, bw, st = _run(insts, K, dtype, rhos, alphas, z0=z0, cg_tol=cg)
    assert st["nonfinite"].max() == 0 and st["eig_not_converged"].max() == 0
    _check(batch, fw, loss, bw, insts, rhos, alphas, tol_it, tol_g, every_k=True, z0=z0d, cg_tol=cg)


def test_c1_maxcut_fp64_every_iterate():
    ensure_lib()
    inst = synth.c1_instance()
    K = 100
    rho = synth.default_rho(inst, K)
    alpha = np.full(K, 1.6)
    say("C1 max-cut n=20 fp64 K=100 forward")
    batch, fw, loss, bw, st = _run([inst], K, np.float64, [rho], [alpha], cg_tol=1e-10, grad=False)
    assert st["cg_iters_max"][0] <= 2
    _check(batch, fw, loss, bw, [inst], [rho], [alpha], 1e-9, 1e-8, every_k=True, grad=False)


def test_c2_small_batch_fp32_forward_backward():
    ensure_lib()
    rng = np.random.default_rng(20)
    insts = [x.astype(np.float32) for x in synth.c2_batch(B=4, p_lo=20, p_hi=45, seed=22)]
    K = 20
    rhos, alphas = _stack_hyper(insts, K, rng)
    say(f"C2-like B=4 p={[i.meta['order'] for i in insts]} fp32 K={K}")
    batch, fw, loss, bw, st = _run(insts, K, np.float32, rhos, alphas)
    assert st["nonfinite"].max() == 0
    _check(batch, fw, loss, bw, insts, rhos, alphas, 1e-5, 1e-4, every_k=True)


def test_first_instance_and_forward_only_path_fp64():
    """Regression: the (x, s, y) ping-pong buffers of the reverse pass (and of
    the forward-only path) hold 64-element-aligned parts; with n, m not
    multiples of 64 the first instance of a batch is the one that would see
    an undersized buffer."""
    ensure_lib()
    from paper_2606_13825_amd import CosmoBatch
    rng = np.random.default_rng(61)
    inst = synth.c2_batch(B=1, p_lo=39, p_hi=39, seed=61)[0]
    K = 3
    rhos, alphas = _stack_hyper([inst], K, rng, dtype=np.float64)
    say(f"first-instance gradients fp64 n={inst.n} m={inst.m} K={K}")
    batch, fw, loss, bw, st = _run([inst], K, np.float64, rhos, alphas, cg_tol=1e-13)
    _check(batch, fw, loss, bw, [inst], rhos, alphas, 1e-10, 1e-9, every_k=True)
    rho = torch.from_numpy(rhos[0]).to(DEV)
    alpha = torch.from_numpy(alphas[0].reshape(K, 1)).to(DEV)
    plain = batch.forward(rho, alpha, tape=False)
    torch.cuda.synchronize()
    for a, b in ((plain.x, fw.x), (plain.s, fw.s), (plain.y, fw.y)):
        assert torch.equal(a, b)


def _appb(n, seed):
    """App. B sampler as a conic instance: nonnegative cone on all m = n/2
    rows, q = -P x*; returns the instance and its rho ~ U(0, 1)."""
    from synth.workloads import appb_instance
    P, A, rho, b, xstar = appb_instance(n, np.random.default_rng(seed))
    inst = synth.ConicInstance(P=P.tocsr(), q=-(P @ xstar), A=A.tocsr(), b=b,
                               cones=[synth.Cone("nonneg", A.shape[0])])
    return inst, rho


@pytest.mark.parametrize("n", [1000, 2000])
def test_appb_instances_fp64(n):
    # the linear-solve backward experiment's instances (App. B), two steps
    ensure_lib()
    inst, rho = _appb(n, 30 + n)
    K = 2
    rhos = [np.stack([rho, 0.5 + rho]).astype(np.float64)]
    alphas = [np.array([1.0, 1.6])]
    say(f"App. B n={n} m={inst.m} nnz={inst.A.nnz} fp64 K={K}")
    batch, fw, loss, bw, st = _run([inst], K, np.float64, rhos, alphas, cg_tol=1e-13)
    assert st["cg_not_converged"].max() == 0
    _check(batch, fw, loss, bw, [inst], rhos, alphas, 1e-9, 1e-8, every_k=True)


def test_appb_instance_fp32_cooperative_cg():
    # the configuration the App. B study times: float32, cooperative CG
    # (4 workgroups per CU at most), CG to its precision floor
    ensure_lib()
    from paper_2606_13825_amd import CosmoBatch
    inst, rho = _appb(2000, 40)
    inst = inst.astype(np.float32)
    K = 2
    rhos = [np.stack([rho, 0.5 + rho]).astype(np.float32)]
    alphas = [np.array([1.0, 1.6], np.float32)]
    say(f"App. B n=2000 fp32 cooperative K={K}")
    batch = CosmoBatch([inst], K=K, dtype=torch.float32, device=DEV, cg_tol=1e-10)
    batch.set_pcg_form(4)
    r = torch.from_numpy(rhos[0]).to(DEV)
    a = torch.from_numpy(alphas[0].reshape(K, 1)).to(DEV)
    stats = batch.new_stats()
    fw = batch.forward(r, a, stats=stats)
    loss, g = batch.residual_loss(fw.x, fw.s, fw.y)
    bw = batch.backward(r, a, fw.tape, *g, stats=stats)
    torch.cuda.synchronize()
    assert batch.stats_dict(stats)["nonfinite"].max() == 0
    _check(batch, fw, loss, bw, [inst], rhos, alphas, 1e-5, 1e-4, every_k=True)
