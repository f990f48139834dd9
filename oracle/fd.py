"""Central finite differences of the unrolled loss (test infrastructure).

Directions are drawn per parameter group (penalties, relaxations, x0, s0,
y0).  A difference quotient is only meaningful on one smooth piece of the
projections, so the active pattern (nonnegative signs, SOC case, PSD inertia)
of every step is recorded at theta + h d and theta - h d and the direction is
redrawn when they differ.
"""
import numpy as np

from .cones import active_signature
from .cosmo import residual_loss, residual_loss_grad, unroll_backward, unroll_forward


def fd_directional(fun, h: float):
    """(f(+h) - f(-h)) / 2h for a scalar function of the step size."""
    return (fun(h) - fun(-h)) / (2.0 * h)


def _signature(inst, tape):
    return tuple(active_signature(st["v"], inst.cones) for st in tape)


def fd_check_unroll(inst, rho, alpha, x0, s0, y0, rng, ndirs=3, h=1e-6, sigma=1e-6,
                    groups=("rho", "alpha", "x0", "s0", "y0"), max_redraw=20):
    """Compare the analytic directional derivative of the final-residual loss
    through K steps with central differences.  Returns a list of
    (group, analytic, finite_difference)."""
    tape, (xK, sK, yK) = unroll_forward(inst, rho, alpha, x0, s0, y0, sigma)
    gx, gs, gy = residual_loss_grad(inst, xK, sK, yK)
    grho, galpha, gx0, gs0, gy0 = unroll_backward(inst, tape, gx, gs, gy, sigma)
    grads = dict(rho=grho, alpha=galpha, x0=gx0, s0=gs0, y0=gy0)
    base = dict(rho=rho, alpha=alpha, x0=x0, s0=s0, y0=y0)
    out = []
    for g in groups:
        done = 0
        for _ in range(max_redraw):
            if done >= ndirs:
                break
            d = rng.standard_normal(np.shape(base[g]))
            if g == "rho":
                d = d * rho              # relative perturbation keeps rho > 0

            def run(t):
                p = dict(base)
                p[g] = base[g] + t * d
                tp, (x, s, y) = unroll_forward(inst, p["rho"], p["alpha"], p["x0"], p["s0"],
                                               p["y0"], sigma)
                return tp, residual_loss(inst, x, s, y)

            tp_p, fp = run(h)
            tp_m, fm = run(-h)
            if _signature(inst, tp_p) != _signature(inst, tp_m):
                continue
            out.append((g, float(np.sum(grads[g] * d)), (fp - fm) / (2.0 * h)))
            done += 1
    return out
