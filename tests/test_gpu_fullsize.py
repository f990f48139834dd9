"""Full-size workloads in the launch configuration bench.py times (the same
batch, K, dtype, hyperparameters and autotuned CG schedule), checked on
sampled outputs the float64 oracle can compute one by one:

  * c2 (64 max-cut SDPs, K = 50, the benchmark's headline workload): every
    step of sampled instances -- the forward step from the GPU's own iterate
    (one-step parity), the whole reverse pass over the GPU's own forward
    record, and the whole trajectory against the oracle's own run;

  * c5 (128 covariance-steering SDPs, K = 30): whole trajectories and
    gradients of two sampled instances (the largest, and the first);
  * c4 (256 Huber SOCPs, K = 40, float64 iterations with the design block
    stored as float32): whole trajectories and gradients of two sampled
    instances, and one-step parity at sampled steps;
  * c3 (32 Lovasz SDPs, K = 50), whose full oracle runs take minutes per
    instance: one-step parity of the forward at sampled steps (the oracle
    started from the GPU's own iterate), and the gradients of the last
    steps, reverse mode in the oracle from the GPU's own iterates and loss
    seeds (those gradients depend on nothing earlier), both at the GPU's own
    taped solves and against exact solves with a floor for the float32
    rounding of the stored steps.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.cones import proj_cone
from gpu_common import (assert_blocks_close, assert_close, ensure_lib, floor_bars, floor_of, one_step_err,
                        oracle_run, say)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _bench_run(name):
    """The benchmark's own workload, hyperparameters and launch configuration:
    one forward + loss + backward pass."""
    import bench
    from paper_2606_13825_amd import CosmoBatch
    wl = bench._workload(name)
    rhos, alphas = bench._hyper(wl)
    kw = {k: wl[k] for k in ("cg_tol", "cg_max_iter", "dense_f32") if k in wl}
    tdt = torch.float32 if wl["dtype"] == "f32" else torch.float64
    batch = CosmoBatch(wl["insts"], K=wl["K"], dtype=tdt, device=DEV, **kw)
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(DEV)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(DEV)
    form, ms = batch.autotune(rho, alpha)
    say(f"{wl['name']}: B={len(wl['insts'])} K={wl['K']} CG schedule {form} ({ms})")
    stats = batch.new_stats()
    fw = batch.forward(rho, alpha, stats=stats)
    _, g = batch.residual_loss(fw.x, fw.s, fw.y)
    bw = batch.backward(rho, alpha, fw.tape, *g, stats=stats)
    torch.cuda.synchronize()
    st = batch.stats_dict(stats)
    say(f"  CG: max iterations {int(st['cg_iters_max'].max())}, total {int(st['cg_iters_total'].sum())}, "
        f"solves not at tolerance {int(st['cg_not_converged'].sum())}")
    assert st["nonfinite"].max() == 0
    return wl, rhos, alphas, batch, fw, bw


def _iterate(batch, fw, i, k):
    x, s, y = batch.tape_iterate(fw.tape, k)[:3]
    return (x[batch.n_off[i]:batch.n_off[i + 1]].double().cpu().numpy(),
            s[batch.m_off[i]:batch.m_off[i + 1]].double().cpu().numpy(),
            y[batch.m_off[i]:batch.m_off[i + 1]].double().cpu().numpy())


def _check_one_steps(wl, rhos, alphas, batch, fw, samples):
    worst = 0.0
    for i, k in samples:
        inst = wl["insts"][i]
        try:
            e, _ = one_step_err(inst, _iterate(batch, fw, i, k), _iterate(batch, fw, i, k + 1), rhos[i][k],
                                alphas[i][k], floor_of(inst))
        except AssertionError as err:
            raise AssertionError(f"instance {i}, step {k}: {err}") from None
        worst = max(worst, e)
    where = samples if len(samples) <= 8 else f"{len(samples)} steps"
    say(f"  one-step parity at {where}: worst rel err {worst:.2e}")


def _step_at(inst, z, rho, alpha, fwd=None, round32=False, resid=0.0, rng=None):
    """The oracle's record of step k from iterate z.  With fwd = (x~, s~, s+)
    (the GPU's taped solve and next slack) the record is rebuilt around
    those values: s^, v and the cone data follow from them by the oracle's
    own formulas.  With round32 the quantities a float32 pipeline stores
    are rounded.  With resid > 0 the solve is replaced by x~ + M^-1 r for a
    random r of norm resid ||xi|| (an inexact solve at that residual)."""
    st = oracle.step_forward(inst, *z, np.asarray(rho, np.float64), float(alpha))
    if resid > 0:
        r = rng.standard_normal(inst.n)
        r *= resid * np.linalg.norm(st["xi"]) / np.linalg.norm(r)
        xt = st["xt"] + st["lu"].solve(r)
        fwd = (xt, inst.b - inst.A @ xt, None)
    if fwd is not None:
        x, s, y = z
        xt, stl, sn = fwd
        sh = st["alpha"] * stl + (1.0 - st["alpha"]) * s
        v = sh + y / st["rho_hat"]
        sn_v, aux = proj_cone(v, inst.cones)
        st.update(xt=xt, st=stl, sh=sh, v=v, sn=sn_v if sn is None else sn, aux=aux)
    if round32:
        for key in ("xt", "st", "sh", "v", "sn"):
            st[key] = st[key].astype(np.float32).astype(np.float64)
    return st


def _reverse(inst, tape, zK):
    gx, gs, gy = oracle.residual_loss_grad(inst, *zK)
    ref_r, ref_a = [], []
    for st in reversed(tape):
        gx, gs, gy, gr, ga = oracle.step_backward(inst, st, gx, gs, gy)
        ref_r.append(gr)
        ref_a.append(ga)
    return np.array(ref_r[::-1]), np.array(ref_a[::-1])


def _check_tail_gradients(wl, rhos, alphas, batch, fw, bw, i, tail, tol, exact=True):
    """grad rho^k and alpha^k of instance i for the last `tail` steps.

    (a) At `tol`: the oracle's reverse pass over the GPU's own iterates,
        taped solves (x~, s~) and next slacks s+ -- the reverse arithmetic,
        adjoint solves and cone VJPs, on the same forward quantities (the
        rho gradient carries s^ - s+, which a single float32 rounding of s+
        already moves by ~1e-4 at this depth).
    (b) grad rho against the oracle's own forward (exact solves), at `tol`
        with a floor: these gradients carry differences such as s~ - s and
        s^ - s+, small near a fixed point, so they move with the forward
        solve's accuracy.  A solve whose residual is 1e-7 ||xi|| (about
        three times the smallest true residual a float32 CG reaches on
        these systems; the paper's tolerance is 1e-8) moves them by d_cg,
        and rounding the stored per-step quantities to float32 by d_32
        (both computed here); the bar allows 4 max(d_cg, d_32).  grad alpha
        is a single dot product over those same differences per step; it
        is checked by (a)."""
    inst, K = wl["insts"][i], wl["K"]
    ks = range(K - tail, K)
    zs = [_iterate(batch, fw, i, k) for k in ks]
    zK = _iterate(batch, fw, i, K)
    fwd = []
    for j, k in enumerate(ks):
        xt, stl = batch.tape_iterate(fw.tape, k)[3:]
        fwd.append((xt[batch.n_off[i]:batch.n_off[i + 1]].double().cpu().numpy(),
                    stl[batch.m_off[i]:batch.m_off[i + 1]].double().cpu().numpy(),
                    (zs[j + 1] if j + 1 < len(zs) else zK)[1]))
    sl_m = slice(batch.m_off[i], batch.m_off[i + 1])
    g_r = bw.grho[K - tail:, sl_m].double().cpu().numpy()
    g_a = bw.galpha[K - tail:, i].double().cpu().numpy()
    at_r, at_a = _reverse(inst, [_step_at(inst, z, rhos[i][k], alphas[i][k], f) for z, k, f in zip(zs, ks, fwd)], zK)
    e1 = assert_close(g_r, at_r, tol, 0.0, f"inst {i} grad rho tail at the GPU's solves")
    e2 = assert_close(g_a, at_a, tol, 0.0, f"inst {i} grad alpha tail at the GPU's solves")
    if not exact:
        say(f"  gradients of the last {tail} steps, instance {i}: at the GPU's solves rel err {max(e1, e2):.2e}")
        return
    ref_r, ref_a = _reverse(inst, [_step_at(inst, z, rhos[i][k], alphas[i][k]) for z, k in zip(zs, ks)], zK)
    r32_r, _ = _reverse(inst, [_step_at(inst, z, rhos[i][k], alphas[i][k], round32=True) for z, k in zip(zs, ks)], zK)
    rng = np.random.default_rng(1000 + i)
    cg_r, _ = _reverse(inst, [_step_at(inst, z, rhos[i][k], alphas[i][k], resid=1e-7, rng=rng)
                              for z, k in zip(zs, ks)], zK)
    d = max(np.linalg.norm(r32_r - ref_r), np.linalg.norm(cg_r - ref_r))
    nref = np.linalg.norm(ref_r)
    xerr = []
    for z, k, f in zip(zs, ks, fwd):
        st = oracle.step_forward(inst, *z, np.asarray(rhos[i][k], np.float64), float(alphas[i][k]))
        xerr.append(np.linalg.norm(f[0] - st["xt"]) / np.linalg.norm(st["xt"]))
    say(f"  gradients of the last {tail} steps, instance {i}: at the GPU's solves rel err {max(e1, e2):.2e}; "
        f"grad rho vs exact solves {np.linalg.norm(g_r - ref_r) / nref:.2e} (d_32 "
        f"{np.linalg.norm(r32_r - ref_r) / nref:.2e}, d_cg {np.linalg.norm(cg_r - ref_r) / nref:.2e}), "
        f"grad alpha vs exact solves {np.linalg.norm(g_a - ref_a) / np.linalg.norm(ref_a):.2e}; "
        f"x~ vs exact solves per step {['%.1e' % e for e in xerr]}")
    assert_close(g_r, ref_r, tol, 4 * d / tol, f"inst {i} grad rho tail")


def _check_whole_run(wl, rhos, alphas, batch, fw, bw, i):
    """Final iterates and all K steps' gradients of instance i against the
    oracle's own float64 run, at the contract bars (1e-5, 1e-4) or twice the
    instance's float32 floor, whichever is larger (gpu_common), array by
    array and, for the slacks and duals, cone block by cone block.  Returns
    (iterate error, gradient error, floors)."""
    inst = wl["insts"][i]
    r64, a64 = rhos[i].astype(np.float64), alphas[i].astype(np.float64)
    ref = oracle_run(inst, r64, a64)
    runs = []
    if wl["dtype"] == "f32":
        # max-cut's M is diagonal (exact solves); the other families run the CG
        cg = 0.0 if wl["name"].startswith("maxcut") else wl.get("cg_tol", 1e-8)
        b_it, b_g, f = floor_bars(inst, r64, a64, ref, cg_tol=cg, runs=runs)
    else:
        b_it, b_g, f = 1e-5, 1e-4, (0.0, 0.0)
    fl = floor_of(inst)
    sl_n = slice(batch.n_off[i], batch.n_off[i + 1])
    sl_m = slice(batch.m_off[i], batch.m_off[i + 1])
    e = [assert_close(a.double().cpu().numpy(), r, b_it, fl, f"inst {i} final {nm}")
         for nm, a, r in (("x", fw.x[sl_n], ref["x"]), ("s", fw.s[sl_m], ref["s"]), ("y", fw.y[sl_m], ref["y"]))]
    e += [assert_blocks_close(a.double().cpu().numpy(), r, inst, 1e-5, f"inst {i} final {nm}", floor=fl,
                              floor_runs=[run[j] for run in runs])
          for j, nm, a, r in ((1, "s", fw.s[sl_m], ref["s"]), (2, "y", fw.y[sl_m], ref["y"]))]
    g = [assert_close(bw.grho[:, sl_m].double().cpu().numpy(), ref["grho"], b_g, 0.0, f"inst {i} grad rho"),
         assert_close(bw.galpha[:, i].double().cpu().numpy(), ref["galpha"], b_g, 0.0, f"inst {i} grad alpha")]
    return max(e), max(g), f


def test_c2_maxcut_full_batch_sampled_instances():
    """Iterates: every one-step check at 1e-5.  Gradients: the oracle's
    reverse pass over the GPU's own forward record (iterates, solves, next
    slacks) at 1e-4 for all 50 steps.  Against the oracle's own float64
    trajectory the final iterates and the gradients are held to the contract
    bars or twice the instance's float32 floor (the oracle's rounding model;
    on some instances of this batch float32 storage alone moves the
    gradients by 1e-4 and more)."""
    ensure_lib()
    wl, rhos, alphas, batch, fw, bw = _bench_run("c2")
    insts, K = wl["insts"], wl["K"]
    orders = [inst.cones[-1].size for inst in insts]
    # the benchmark's oracle sample (the first 16 instances) and the extreme orders
    for i in sorted(set(range(16)) | {int(np.argmax(orders)), int(np.argmin(orders))}):
        inst = insts[i]
        _check_one_steps(wl, rhos, alphas, batch, fw, [(i, k) for k in range(K)])
        _check_tail_gradients(wl, rhos, alphas, batch, fw, bw, i, K, 1e-4, exact=False)
        e, g, f = _check_whole_run(wl, rhos, alphas, batch, fw, bw, i)
        say(f"  instance {i} (p={orders[i]}): final iterates vs the oracle's run {e:.2e}, gradients {g:.2e} "
            f"(float32 floor {f[0]:.1e}, {f[1]:.1e})")


def test_c5_covsteer_full_batch_sampled_instances():
    ensure_lib()
    wl, rhos, alphas, batch, fw, bw = _bench_run("c5")
    insts = wl["insts"]
    largest = int(np.argmax([inst.n for inst in insts]))
    for i in sorted({0, largest}):
        inst = insts[i]
        e, g, f = _check_whole_run(wl, rhos, alphas, batch, fw, bw, i)
        say(f"  instance {i} (n={inst.n}, m={inst.m}): final iterates {e:.2e}, gradients {g:.2e} "
            f"(float32 floor {f[0]:.1e}, {f[1]:.1e})")


def test_c3_lovasz_full_batch_sampled_steps():
    ensure_lib()
    wl, rhos, alphas, batch, fw, bw = _bench_run("c3")
    K, B = wl["K"], len(wl["insts"])
    big = int(np.argmax([inst.meta["order"] for inst in wl["insts"]]))
    _check_one_steps(wl, rhos, alphas, batch, fw, [(0, 0), (big, 0), (big, K // 2), (big, K - 3), (big, K - 2),
                                                   (B - 1, K - 1)])
    _check_tail_gradients(wl, rhos, alphas, batch, fw, bw, big, 3, 1e-4)
    # whole trajectories: this family's float32 floor is large (its iterates
    # shrink by four orders of magnitude over the unroll while the rounding
    # of the early, large ones stays), and the bars follow it
    for i in (0, big):
        e, g, f = _check_whole_run(wl, rhos, alphas, batch, fw, bw, i)
        say(f"  instance {i} (order {wl['insts'][i].meta['order']}): final iterates {e:.2e}, gradients {g:.2e} "
            f"(float32 floor {f[0]:.1e}, {f[1]:.1e})")


def test_c4_huber_full_batch_sampled_instances():
    """The benchmark's line: float64 iterations on float32 data, the design
    block stored as float32 (lossless).  Whole trajectories and gradients of
    two sampled instances against the oracle's own float64 runs at the
    contract bars, plus one-step parity at sampled steps."""
    ensure_lib()
    wl, rhos, alphas, batch, fw, bw = _bench_run("c4")
    K, B = wl["K"], len(wl["insts"])
    assert batch.n_dense == B and batch.dense_val.dtype == torch.float32
    _check_one_steps(wl, rhos, alphas, batch, fw, [(0, 0), (B - 1, K // 2), (B // 2, K - 1)])
    for i in (0, B - 1):
        e, g, _ = _check_whole_run(wl, rhos, alphas, batch, fw, bw, i)
        say(f"  instance {i}: final iterates vs the oracle's run {e:.2e}, gradients {g:.2e}")
