"""Shared pieces of the GPU parity tests: running the float64 oracle on the
same (rounded) data and hyperparameters, and the norm-wise tolerance test.

Tolerance (per instance and per array): ||gpu - ref||_2 <= tol * max(||ref||_2, floor)
with floor = 1e-6 max(1, ||b||, ||q||), so arrays whose reference is ~0 are
compared against the data scale.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402


def say(msg: str) -> None:
    print(msg, flush=True)


def ensure_lib():
    from paper_2606_13825_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        raise RuntimeError("libcosmo_unroll.so is not built; run __graft_entry__.build() first")


def floor_of(inst) -> float:
    return 1e-6 * max(1.0, float(np.linalg.norm(inst.b)), float(np.linalg.norm(inst.q)))


def rel_err(gpu, ref, floor=0.0) -> float:
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(gpu - ref) / max(np.linalg.norm(ref), floor, 1e-300))


def assert_close(gpu, ref, tol, floor, what):
    e = rel_err(gpu, ref, floor)
    assert np.all(np.isfinite(np.asarray(gpu))), f"{what}: non-finite values"
    assert e <= tol, f"{what}: relative error {e:.3e} > {tol:.1e}"
    return e


def oracle_run(inst, rho_k_m, alpha_k, with_grad=True, x0=None, s0=None, y0=None):
    """Forward (and loss-gradient backward) of one instance in float64."""
    tape, (x, s, y) = oracle.unroll_forward(inst, rho_k_m, alpha_k, x0, s0, y0)
    out = dict(tape=tape, x=x, s=s, y=y, loss=oracle.residual_loss(inst, x, s, y))
    if with_grad:
        g = oracle.residual_loss_grad(inst, x, s, y)
        grho, galpha, gx0, gs0, gy0 = oracle.unroll_backward(inst, tape, *g)
        out.update(grho=grho, galpha=galpha, gx0=gx0, gs0=gs0, gy0=gy0)
    return out


def one_step_err(inst, z, z_next, rho_k, alpha_k, fl, tol=1e-5):
    """The float64 oracle's step from the GPU's iterate z = (x, s, y) against
    the GPU's next iterate, per array, at `tol` relative, with one floor: the
    step may carry the effect of 8 float32 roundings of the right-hand side xi
    through the solve, M^-1 (fl32(xi) - xi), and on to s and y (the
    projection is nonexpansive, y+ adds rho (s^ - s+)).  The library keeps xi
    in float64; the floor stands in for the float32 rounding of the stored
    per-step values (s~, s^, v), which reach the next iterate the same way.
    Returns (worst error, number of arrays where the floor decided)."""
    x, s, y = z
    st = oracle.step_forward(inst, x, s, y, np.asarray(rho_k, np.float64), float(alpha_k))
    dxt = st["lu"].solve(st["xi"].astype(np.float32).astype(np.float64) - st["xi"])
    dsh = float(alpha_k) * np.linalg.norm(inst.A @ dxt)
    floors = {"x": 8 * float(alpha_k) * np.linalg.norm(dxt), "s": 8 * dsh,
              "y": 16 * float(st["rho_hat"].max()) * dsh}
    worst, n_floor = 0.0, 0
    for nm, g, r in (("x", z_next[0], st["xn"]), ("s", z_next[1], st["sn"]), ("y", z_next[2], st["yn"])):
        f = max(fl, floors[nm] / tol)
        n_floor += f > np.linalg.norm(r)
        worst = max(worst, assert_close(g, r, tol, f, nm))
    return worst, n_floor


# ---- float32 bars from measured floors ------------------------------------
#
# A float32 pipeline stores every per-step value in float32 and stops its
# solves at a float32 residual.  How far that alone moves a K-step
# trajectory and its gradients depends on the instance (some families
# amplify it a thousandfold: their iterates shrink by orders of magnitude
# while the rounding of the early, large ones stays), so each checked
# instance gets its floor measured by the oracle's rounding model
# (unroll_forward with store_dtype): the largest error, against the exact
# float64 run, of three realisations -- values rounded to nearest with exact
# solves, and two with every stored value moved by up to one unit in the last
# place and solves stopped at the run's CG residual.  The bar is the
# contract's (1e-5 iterates, 1e-4 gradients) or FLOOR_FACTOR times that
# floor, whichever is larger.
FLOOR_FACTOR = 2.0
FLOAT32_CG_RESID = 1e-7   # where a float32 CG's true residual stops, at the smallest


def fp32_floor(inst, rho_k_m, alpha_k, ref, x0=None, s0=None, y0=None, with_grad=True, cg_tol=0.0, runs=None):
    """(iterate floor, gradient floor) of one instance against its float64 run
    `ref` (oracle_run's output), per array, the largest over the model's
    realisations (oracle.rounding_floor_runs); cg_tol = 0: the pipeline's
    solves are exact (diagonal M).  runs: a list that receives each
    realisation's final (x, s, y)."""
    resid = max(cg_tol, FLOAT32_CG_RESID) if cg_tol > 0 else 0.0
    fl = floor_of(inst)
    e_it = e_g = 0.0
    for x, s, y, grho, galpha in oracle.rounding_floor_runs(inst, rho_k_m, alpha_k, x0, s0, y0,
                                                            backward=with_grad, solve_resid=resid):
        if runs is not None:
            runs.append((x, s, y))
        e_it = max([e_it] + [rel_err(a, ref[k], fl) for a, k in ((x, "x"), (s, "s"), (y, "y"))])
        if with_grad:
            e_g = max(e_g, rel_err(grho, ref["grho"]), rel_err(galpha, ref["galpha"]))
    return e_it, e_g


def floor_bars(inst, rho_k_m, alpha_k, ref, tol_it=1e-5, tol_g=1e-4, **kw):
    """(iterate bar, gradient bar, (iterate floor, gradient floor)); kw as
    fp32_floor's."""
    f_it, f_g = fp32_floor(inst, rho_k_m, alpha_k, ref, **kw)
    return max(tol_it, FLOOR_FACTOR * f_it), max(tol_g, FLOOR_FACTOR * f_g), (f_it, f_g)


def _row_blocks(inst):
    """Row ranges of the cone blocks (zero and nonnegative rows one block each)."""
    out, r = [], 0
    for c in inst.cones:
        n = c.size * (c.size + 1) // 2 if c.kind == "psd" else c.size
        out.append((r, r + n))
        r += n
    return out


def assert_blocks_close(gpu, ref, inst, tol, what, rel_floor=1e-3, floor=0.0, floor_runs=()):
    """Per cone block: ||gpu - ref||_blk <= bar max(||ref||_blk, rel_floor
    ||ref||, floor), so one wrong block among hundreds is not diluted by the
    others (a block with a negligible share of the array is measured against
    rel_floor of the whole).  bar: tol, or FLOOR_FACTOR times the same block's
    error in the floor realisations `floor_runs` (arrays like ref), whichever
    is larger."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    whole = np.linalg.norm(ref)
    worst = 0.0
    for a, b in _row_blocks(inst):
        den = max(np.linalg.norm(ref[a:b]), rel_floor * whole, floor, 1e-300)
        bar = max([tol] + [FLOOR_FACTOR * np.linalg.norm(np.asarray(f)[a:b] - ref[a:b]) / den for f in floor_runs])
        e = np.linalg.norm(gpu[a:b] - ref[a:b]) / den
        assert e <= bar, f"{what}: rows {a}:{b} relative error {e:.3e} > {bar:.1e}"
        worst = max(worst, e)
    return worst
