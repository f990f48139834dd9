"""Dense sub-blocks of A (cosmo_dense_block) on the GPU: the unroll with a
block given once as a dense array -- fused into the CG operator, and applied
by the dense row / column products everywhere else -- matches the float64
oracle, which only ever sees A as one sparse matrix, and matches the same
batch passed as CSR alone.

Cases: uneven batches mixing instances with and without a dense block;
widths that are not a multiple of the 16-byte piece nor of the 64-lane strip
(ragged tails); row counts not a multiple of a workgroup's rows; one to
four placements with scales other than +-1; float64 and float32; float32
storage of the blocks in a float64 batch."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import synth
from synth import Cone, ConicInstance
from gpu_common import assert_close, ensure_lib, floor_of, oracle_run, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _stacked_instance(rng, rows, cols, scales, n_extra=5, soc=(4, 3)):
    """A nonnegative-and-SOC program whose A holds one dense G at len(scales)
    row offsets (scale_p G), plus a sparse identity part on extra variables
    and SOC rows on the G columns; P diagonal and positive."""
    G = rng.standard_normal((rows, cols))
    npl = len(scales)
    n = cols + n_extra
    blocks = [sp.hstack([sc * sp.csr_matrix(G), sp.csr_matrix((rows, n_extra))]) for sc in scales]
    extra = sp.hstack([sp.csr_matrix((n_extra, cols)), sp.identity(n_extra)])
    srows, scols, svals, sb = [], [], [], []
    r = 0
    for d in soc:
        sel = rng.choice(cols, size=d - 1, replace=False)
        sb.append(1.0)
        for t, g in enumerate(sel):
            srows.append(r + 1 + t)
            scols.append(int(g))
            svals.append(-1.0)
            sb.append(0.0)
        r += d
    socA = sp.csr_matrix((svals, (srows, scols)), shape=(r, n))
    A = sp.vstack(blocks + [extra, socA]).tocsr()
    m = A.shape[0]
    b = np.concatenate([rng.standard_normal(npl * rows + n_extra), np.array(sb)])
    P = sp.diags(rng.uniform(0.5, 2.0, n)).tocsr()
    q = rng.standard_normal(n)
    cones = [Cone("nonneg", npl * rows + n_extra)] + [Cone("soc", d) for d in soc]
    inst = ConicInstance(P, q, A, b, cones,
                         {"dense": {"col0": 0, "rows": rows, "cols": cols,
                                    "place": [(p * rows, float(sc)) for p, sc in enumerate(scales)]}})
    inst.check()
    assert A.shape == (m, n)
    return inst


def _batch(dtype):
    rng = np.random.default_rng(31)
    insts = [_stacked_instance(rng, 70, 37, (1.0, -1.0)),          # ragged width, two placements
             synth.huber_socp(rng, n_obs=130, n_coef=61, n_soc=6),  # the Huber form, 61 columns
             _stacked_instance(rng, 65, 300, (1.0, -0.5, 2.0)),     # three placements, width > one strip
             _stacked_instance(rng, 33, 8, (1.0,)),                 # one placement
             _stacked_instance(rng, 41, 23, (1.0, -1.0, 0.5, -2.0))]  # the most placements a block may have
    plain = synth.huber_socp(rng, n_obs=40, n_coef=9, n_soc=2)
    plain.meta.pop("dense")                                         # an instance given as CSR alone
    insts.insert(2, plain)
    return [x.astype(dtype) for x in insts]


def _run(insts, K, dtype, rhos, alphas, dense, cg_tol, dense_f32=False):
    from paper_2606_13825_amd import CosmoBatch
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    batch = CosmoBatch(insts, K=K, dtype=tdt, device=DEV, cg_tol=cg_tol, cg_max_iter=2000, dense=dense,
                       dense_f32=dense_f32)
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(DEV)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(DEV)
    stats = batch.new_stats()
    fw = batch.forward(rho, alpha, stats=stats)
    loss, g = batch.residual_loss(fw.x, fw.s, fw.y)
    bw = batch.backward(rho, alpha, fw.tape, *g, stats=stats)
    torch.cuda.synchronize()
    st = batch.stats_dict(stats)
    assert st["nonfinite"].max() == 0
    return batch, fw, loss, bw


def _hyper(insts, K, dtype, seed=5):
    rng = np.random.default_rng(seed)
    rhos, alphas = [], []
    for inst in insts:
        r, a = synth.perturbed_hyper(inst, K, rng)
        rhos.append(r.astype(dtype))
        alphas.append(a.astype(dtype))
    return rhos, alphas


@pytest.mark.parametrize("dtype,tol_it,tol_g,cg_tol", [(np.float64, 1e-9, 1e-8, 1e-13),
                                                       (np.float32, 1e-5, 1e-4, 1e-10)])
def test_dense_blocks_every_iterate_and_gradients(dtype, tol_it, tol_g, cg_tol):
    ensure_lib()
    insts = _batch(dtype)
    K = 5
    rhos, alphas = _hyper(insts, K, dtype)
    say(f"dense blocks {np.dtype(dtype).name}: B={len(insts)} shapes {[x.A.shape for x in insts]} K={K}")
    batch, fw, loss, bw = _run(insts, K, dtype, rhos, alphas, True, cg_tol)
    assert batch.n_dense == 5
    worst_it = worst_g = 0.0
    for i, inst in enumerate(insts):
        ref = oracle_run(inst, rhos[i].astype(np.float64), alphas[i].astype(np.float64))
        fl = floor_of(inst)
        sl_n = slice(batch.n_off[i], batch.n_off[i + 1])
        sl_m = slice(batch.m_off[i], batch.m_off[i + 1])
        for k in range(1, K + 1):
            x, s, y, _, _ = batch.tape_iterate(fw.tape, k)
            st = ref["tape"][k - 1]
            for nm, g_, r_ in (("x", x[sl_n], st["xn"]), ("s", s[sl_m], st["sn"]), ("y", y[sl_m], st["yn"])):
                worst_it = max(worst_it, assert_close(g_.double().cpu().numpy(), r_, tol_it, fl,
                                                      f"inst {i} iterate {nm}^{k}"))
        assert abs(float(loss[i]) - ref["loss"]) <= tol_g * abs(ref["loss"])
        for nm, g_, r_ in (("grad rho", bw.grho[:, sl_m], ref["grho"]), ("grad alpha", bw.galpha[:, i], ref["galpha"]),
                           ("grad x0", bw.gx0[sl_n], ref["gx0"]), ("grad s0", bw.gs0[sl_m], ref["gs0"]),
                           ("grad y0", bw.gy0[sl_m], ref["gy0"])):
            worst_g = max(worst_g, assert_close(g_.double().cpu().numpy(), r_, tol_g, 0.0, f"inst {i} {nm}"))
    say(f"  worst iterate error {worst_it:.2e}, worst gradient error {worst_g:.2e}")


def test_float32_stored_blocks_in_a_float64_batch():
    """Data that are float32 numbers (generated in float64, rounded), a
    float64 batch whose dense blocks are stored as float32: every iterate
    and gradient at the float64 bars, and the same as the all-float64 CSR
    path up to the order of the sums.  Blocks whose values are not float32
    numbers are refused by the binding."""
    ensure_lib()
    from paper_2606_13825_amd import CosmoBatch
    insts = [x.astype(np.float32).astype(np.float64) for x in _batch(np.float64)]
    K = 4
    rhos, alphas = _hyper(insts, K, np.float64, seed=8)
    say(f"float32-stored dense blocks in a float64 batch: B={len(insts)} K={K}")
    b1, f1, l1, g1 = _run(insts, K, np.float64, rhos, alphas, True, 1e-13, dense_f32=True)
    b2, f2, l2, g2 = _run(insts, K, np.float64, rhos, alphas, False, 1e-13)
    assert b1.n_dense == 5 and b1.dense_val.dtype == torch.float32
    for a, b in ((f1.x, f2.x), (f1.s, f2.s), (f1.y, f2.y), (l1, l2), (g1.grho, g2.grho), (g1.galpha, g2.galpha),
                 (g1.gx0, g2.gx0), (g1.gs0, g2.gs0), (g1.gy0, g2.gy0)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-10 * max(np.linalg.norm(b), 1e-30)
    worst = 0.0
    for i, inst in enumerate(insts):
        ref = oracle_run(inst, rhos[i], alphas[i])
        fl = floor_of(inst)
        sl_n = slice(b1.n_off[i], b1.n_off[i + 1])
        sl_m = slice(b1.m_off[i], b1.m_off[i + 1])
        for nm, g_, r_, tol, f in (("x", f1.x[sl_n], ref["x"], 1e-9, fl), ("s", f1.s[sl_m], ref["s"], 1e-9, fl),
                                   ("y", f1.y[sl_m], ref["y"], 1e-9, fl),
                                   ("grad rho", g1.grho[:, sl_m], ref["grho"], 1e-8, 0.0),
                                   ("grad alpha", g1.galpha[:, i], ref["galpha"], 1e-8, 0.0)):
            worst = max(worst, assert_close(g_.cpu().numpy(), r_, tol, f, f"inst {i} {nm}"))
    say(f"  worst error against the oracle {worst:.2e}")
    with pytest.raises(ValueError):
        CosmoBatch(_batch(np.float64), K=1, dtype=torch.float64, device=DEV, dense_f32=True)


def test_dense_path_equals_csr_path_fp64():
    """The same batch with the dense blocks given as CSR: only the order of
    the sums differs."""
    ensure_lib()
    insts = _batch(np.float64)
    K = 4
    rhos, alphas = _hyper(insts, K, np.float64, seed=6)
    b1, f1, l1, g1 = _run(insts, K, np.float64, rhos, alphas, True, 1e-13)
    b2, f2, l2, g2 = _run(insts, K, np.float64, rhos, alphas, False, 1e-13)
    assert b1.n_dense == 5 and b2.n_dense == 0
    assert b1.A_nnz < b2.A_nnz
    for a, b in ((f1.x, f2.x), (f1.s, f2.s), (f1.y, f2.y), (l1, l2), (g1.grho, g2.grho), (g1.galpha, g2.galpha),
                 (g1.gx0, g2.gx0), (g1.gs0, g2.gs0), (g1.gy0, g2.gy0)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-10 * max(np.linalg.norm(b), 1e-30)


def test_dense_block_rows_a_workgroup_multiple_and_graph_replay():
    """Rows that fill whole workgroups of the row products (128 = 2 x 64),
    width 256 (exactly one strip), and the same unroll replayed from a graph:
    bitwise equal to the eager launches."""
    ensure_lib()
    from paper_2606_13825_amd import CosmoBatch
    rng = np.random.default_rng(41)
    insts = [_stacked_instance(rng, 128, 256, (1.0, -1.0)).astype(np.float32),
             _stacked_instance(rng, 64, 4, (1.0, -1.0)).astype(np.float32)]
    K = 3
    rhos, alphas = _hyper(insts, K, np.float32, seed=7)
    batch = CosmoBatch(insts, K=K, dtype=torch.float32, device=DEV, cg_tol=1e-10, cg_max_iter=2000)
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(DEV)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(DEV)
    tape, ws = batch.new_tape(), batch.new_fwd_ws()
    out = tuple(torch.empty(n, device=DEV) for n in (batch.n_tot, batch.m_tot, batch.m_tot))
    eager = batch.forward(rho, alpha, tape=tape, ws=ws, out=out)
    ref = [t.clone() for t in (eager.x, eager.s, eager.y)]
    batch.set_graph(True)
    for rep in range(3):
        fw = batch.forward(rho, alpha, tape=tape, ws=ws, out=out)
        torch.cuda.synchronize()
        for a, b in zip((fw.x, fw.s, fw.y), ref):
            assert torch.equal(a, b), f"graph replay {rep} differs"
    for i, inst in enumerate(insts):
        o = oracle_run(inst, rhos[i].astype(np.float64), alphas[i].astype(np.float64), with_grad=False)
        sl_n = slice(batch.n_off[i], batch.n_off[i + 1])
        assert_close(ref[0][sl_n].double().cpu().numpy(), o["x"], 1e-5, floor_of(inst), f"inst {i} final x")


def test_cooperative_form_refused_with_dense_blocks():
    ensure_lib()
    from paper_2606_13825_amd import CosmoBatch
    from paper_2606_13825_amd._lib import CosmoError
    rng = np.random.default_rng(43)
    batch = CosmoBatch([_stacked_instance(rng, 20, 6, (1.0, -1.0)).astype(np.float32)], K=1,
                       dtype=torch.float32, device=DEV)
    with pytest.raises(CosmoError):
        batch.set_pcg_form(2)
    assert batch.pcg_form() == 0
