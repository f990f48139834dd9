"""Graph mode: the unroll recorded into a HIP graph and replayed must give
bitwise the eager result, on every replay, with the program's own eager work
and synchronisations between replays, and after the data behind the
recorded pointers changes.  Two batches: one with a genuine CG (mixed cones)
and one whose PSD order classes run on forked streams (max-cut)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import ensure_lib, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _batches():
    rng = np.random.default_rng(90)
    mixed = [synth.random_mixed(rng, n=20, soc_dims=(3, 4), psd_orders=(3, 5)) for _ in range(3)]
    maxcut = synth.c2_batch(B=6, p_lo=20, p_hi=140, seed=91)
    return {"mixed": mixed, "maxcut": maxcut}


def _hyper(insts, K, seed):
    rng = np.random.default_rng(seed)
    hy = [synth.perturbed_hyper(i, K, rng) for i in insts]
    rho = np.concatenate([h[0] for h in hy], axis=1).astype(np.float32)
    alpha = np.stack([h[1] for h in hy], axis=1).astype(np.float32)
    return torch.from_numpy(rho).to(DEV), torch.from_numpy(alpha).to(DEV)


class _Buffers:
    """Fixed buffers so that every call passes the same pointers."""

    def __init__(self, batch):
        f = lambda n: torch.empty(n, dtype=batch.dtype, device=DEV)
        self.tape, self.fws, self.bws = batch.new_tape(), batch.new_fwd_ws(), batch.new_bwd_ws()
        self.fout = (f(batch.n_tot), f(batch.m_tot), f(batch.m_tot))
        self.bout = (torch.empty((batch.K, batch.m_tot), dtype=batch.dtype, device=DEV),
                     torch.empty((batch.K, batch.B), dtype=batch.dtype, device=DEV),
                     f(batch.n_tot), f(batch.m_tot), f(batch.m_tot))
        self.seeds = (f(batch.n_tot), f(batch.m_tot), f(batch.m_tot))


def _step(batch, buf, rho, alpha):
    fw = batch.forward(rho, alpha, tape=buf.tape, ws=buf.fws, out=buf.fout)
    _, g = batch.residual_loss(fw.x, fw.s, fw.y)
    for dst, src in zip(buf.seeds, g):
        dst.copy_(src)
    bw = batch.backward(rho, alpha, buf.tape, *buf.seeds, ws=buf.bws, out=buf.bout)
    return [t.clone() for t in (fw.x, fw.s, fw.y, bw.grho, bw.galpha, bw.gx0)]


@pytest.mark.parametrize("name", ["mixed", "maxcut"])
def test_graph_replays_match_eager(name):
    ensure_lib()
    from paper_2606_13825_amd import CosmoBatch, psd_proj
    insts = [i.astype(np.float32) for i in _batches()[name]]
    K = 6
    batch = CosmoBatch(insts, K=K, dtype=torch.float32, device=DEV)
    rho, alpha = _hyper(insts, K, 92)
    rho2, alpha2 = _hyper(insts, K, 93)
    buf = _Buffers(batch)
    say(f"graph mode {name}: B={len(insts)} K={K}")
    eager = _step(batch, buf, rho, alpha)
    eager2 = _step(batch, buf, rho2, alpha2)
    torch.cuda.synchronize()
    batch.set_graph(True)
    assert batch.graph()
    side = torch.randn(50 * 51 // 2, device=DEV)
    for rep in range(4):
        r, a, ref = (rho, alpha, eager) if rep % 2 == 0 else (rho2, alpha2, eager2)
        got = _step(batch, buf, r, a)
        torch.cuda.synchronize()
        for u, v in zip(got, ref):
            assert torch.equal(u, v), f"replay {rep} differs from the eager result"
        psd_proj(side, [50])            # eager library work between replays
        torch.cuda.synchronize()
    batch.set_graph(False)
    again = _step(batch, buf, rho, alpha)
    torch.cuda.synchronize()
    for u, v in zip(again, eager):
        assert torch.equal(u, v)


def test_graph_mode_refuses_cooperative_cg():
    ensure_lib()
    from paper_2606_13825_amd import CosmoBatch
    insts = [i.astype(np.float32) for i in _batches()["mixed"]]
    batch = CosmoBatch(insts, K=2, dtype=torch.float32, device=DEV)
    batch.set_graph(True)
    with pytest.raises(RuntimeError, match="cooperative"):
        batch.set_pcg_form(1)
    batch.set_graph(False)
    batch.set_pcg_form(1)
    with pytest.raises(RuntimeError, match="cooperative"):
        batch.set_graph(True)
