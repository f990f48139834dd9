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
