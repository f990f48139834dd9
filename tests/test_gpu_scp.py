"""Sequential convex programming for the unicycle (App. F) with the convex
steps solved on the GPU (paper_2606_13825_amd.scp, batched vanilla COSMO in
float64) against the oracle's SCP (oracle.scp, each step solved by the
float64 oracle COSMO): the same outer iterations, accept/reject decisions,
inner step counts and final trajectory."""
import numpy as np
import pytest
import torch

import oracle.scp
from gpu_common import ensure_lib, say
from synth.covsteer import (unicycle_scenario, unicycle_subproblem, unicycle_initial_reference, unicycle_step,
                            unicycle_jacobians, unpack_solution)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _problem(sc):
    dt = sc["dt"]
    return dict(step=lambda x, u: unicycle_step(x, u, dt), jacobians=lambda x, u: unicycle_jacobians(x, u, dt))


def test_scp_unicycle_matches_the_oracle_fp64():
    ensure_lib()
    from paper_2606_13825_amd.scp import scp_solve, ScpTiming
    scs = [unicycle_scenario(np.random.default_rng(seed), N=4) for seed in (1, 3)]
    tm = ScpTiming()
    # every scenario of the batch shares dt, so one pair of dynamics callables serves all
    got = scp_solve(scs, **_problem(scs[0]), subproblem=unicycle_subproblem, unpack=unpack_solution,
                    reference=unicycle_initial_reference, eps=1e-6, check=1, dtype=torch.float64, device=DEV,
                    cg_tol=1e-12, timing=tm)
    say(f"  rounds {tm.rounds} batch sizes {tm.batch_sizes} solve {tm.solve_s:.2f}s build {tm.build_s:.2f}s")
    for sc, g in zip(scs, got):
        mu0, v0 = unicycle_initial_reference(sc)
        ref = oracle.scp.scp(sc, **_problem(sc), subproblem=unicycle_subproblem, unpack=unpack_solution,
                             mu_ref=mu0, v_ref=v0, eps=1e-6)
        say(f"  gpu outer {g.outer} inner {[h.inner for h in g.history]}")
        say(f"  oracle outer {ref['outer']} inner {[h['inner'] for h in ref['history']]}")
        assert g.converged and ref["converged"]
        assert g.outer == ref["outer"]
        assert [h.accepted for h in g.history] == [h["accepted"] for h in ref["history"]]
        assert [h.inner for h in g.history] == [h["inner"] for h in ref["history"]]
        # the convex solves of the two sides take the same steps and agree to
        # ~1e-8 in the iterate (float64 rounding over ~1000 steps, CG at 1e-12
        # per step); the merit and the model weigh each of the 2 N nx defect or
        # virtual-control entries by lam_nu = 1e4, i.e. ~2.4e-3 on values of
        # at least ~500 near the end: 1e-5 relative
        dphi = max(abs(h.phi_new - r["phi_new"]) / abs(r["phi_new"]) for h, r in zip(g.history, ref["history"]))
        dmod = max(abs(h.model - r["model"]) / abs(r["model"]) for h, r in zip(g.history, ref["history"]))
        dmu = np.abs(g.mu - ref["mu"]).max() / max(1.0, np.abs(ref["mu"]).max())
        dv = np.abs(g.v - ref["v"]).max() / max(1.0, np.abs(ref["v"]).max())
        say(f"  max rel diff: merit {dphi:.2e} model {dmod:.2e} mean {dmu:.2e} feedforward {dv:.2e}")
        assert [h.rho for h in g.history] == [r["rho"] for r in ref["history"]]
        assert dphi <= 1e-5 and dmod <= 1e-5
        assert dmu <= 1e-6 and dv <= 1e-6
        d = np.array([g.mu[t + 1] - unicycle_step(g.mu[t], g.v[t], sc["dt"]) for t in range(sc["N"])])
        assert np.abs(d).max() < 1e-3
