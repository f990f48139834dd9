"""The learned hyperparameter policy inside the unroll, and the log-residual
training loss, in float64 (test infrastructure; see the package doc).

Policy (App. E "Policy Parameterization"; bounds, widths and initial values
from Table 2).  At iterate z^k = (x, s, y), with s^{k-1} and the s~ of the
step that produced z^k:
    KKT residuals  r_p = A x + s - b,          N_p = max(|A x|_inf, |s|_inf, |b|_inf)
                   r_d = P x + q - A' y,       N_d = max(|P x|_inf, |q|_inf, |A' y|_inf)
                   (r_d with the sign of reading R2), normalised rbar = r / N
    ADMM residuals delta_p = s - s~,  delta_d = s - s^{k-1}   (both 0 at k = 0)
    per-row features xi_rho,i = (l_rho,i, s_i, y_i, rbar_p,i, log(|rbar_d|_inf + eps),
                                 delta_p,i, delta_d,i)
    per-instance    xi_alpha  = (l_alpha, log(|rbar_p|_inf + eps), log(|rbar_d|_inf + eps),
                                 log(|delta_p|_inf + eps), log(|delta_d|_inf + eps))
    l^{k+1} = l^k + MLP(xi^k)   (two hidden ReLU layers of 32, scalar output)
    rho^k = exp((log rho_max - log rho_min) sigmoid(l_rho^{k+1}) + log rho_min)
    alpha^k = 2 sigmoid(l_alpha^{k+1})
and (rho^k, alpha^k) drive the step z^k -> z^{k+1} (rho^k rectified inside
the step, as for fixed penalties).  l^0: one learnable logit per cone kind
(zero, nonnegative, second-order, PSD) broadcast over the rows, and one for
alpha.

Loss (the log-residual loss of Sec. "Experiments"):
    L = sum_{k=1..K} log(|r_d^k|^2 / |r_d^0|^2 + |r_p^k|^2 / |r_p^0|^2)
with the denominators held constant (detached).

Reverse mode: each COSMO step by step_backward (which takes the cotangent
the delta_p feature sends to s~); the policy step and the loss terms by
PyTorch's reverse-mode autograd, on the CPU in float64, over plain tensor
ops.  Ties in an infinity norm or in the max of a normaliser therefore split
the cotangent evenly among the tied entries, and |.| has derivative 0 at 0.

Readings (silent passages), listed with the design notes: the feature
ordering and the step indexing above; a zero normaliser N makes rbar = 0
(then r = 0 too) with no gradient through N; a zero loss denominator is
replaced by 1.
"""
import numpy as np
import torch

from .cosmo import step_forward, step_backward

RHO_MIN, RHO_MAX = 1e-3, 1e3          # Table 2 penalty bounds
EPS = 1e-12                           # App. E, inside the logarithms
HIDDEN = 32                           # Table 2: 32 x 32 ReLU MLP
N_FEAT_RHO, N_FEAT_ALPHA = 7, 5
KINDS = ("zero", "nonneg", "soc", "psd")
TABLE2_RHO0 = (100.0, 0.1, 0.1, 0.1)  # initial (rho_eq, rho_ineq, rho_soc, rho_psd)
TABLE2_ALPHA0 = 1.6


def mlp_size(n_in: int) -> int:
    return n_in * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1


PARAM_COUNT = mlp_size(N_FEAT_RHO) + mlp_size(N_FEAT_ALPHA) + len(KINDS) + 1


def unpack(theta):
    """Split the flat parameter vector (numpy or torch) into named parts.
    Layout: the rho MLP, then the alpha MLP, each as W1 [n_in][32]
    (input-major), b1 [32], W2 [32][32] (input-major), b2 [32], w3 [32],
    b3 [1]; then l_rho^0 [4] by cone kind and l_alpha^0 [1]."""
    out, o = {}, 0

    def take(name, *shape):
        nonlocal o
        cnt = int(np.prod(shape)) if shape else 1
        out[name] = theta[o:o + cnt].reshape(shape) if shape else theta[o:o + cnt].reshape(())
        o += cnt

    for pre, n_in in (("r", N_FEAT_RHO), ("a", N_FEAT_ALPHA)):
        take(pre + "W1", n_in, HIDDEN)
        take(pre + "b1", HIDDEN)
        take(pre + "W2", HIDDEN, HIDDEN)
        take(pre + "b2", HIDDEN)
        take(pre + "w3", HIDDEN)
        take(pre + "b3")
    take("l_rho0", len(KINDS))
    take("l_alpha0")
    assert o == PARAM_COUNT
    return out


def logit_of_rho(rho):
    """Inverse of the penalty squashing."""
    t = (np.log(rho) - np.log(RHO_MIN)) / (np.log(RHO_MAX) - np.log(RHO_MIN))
    return np.log(t / (1.0 - t))


def logit_of_alpha(alpha):
    t = alpha / 2.0
    return np.log(t / (1.0 - t))


def init_params(rng: np.random.Generator, head_scale: float = 0.0) -> np.ndarray:
    """First two layers ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)); the last layer
    zero (App. E's initialisation: the untrained policy is COSMO with fixed
    penalties) unless head_scale > 0, which draws it from U(-head_scale,
    head_scale); l^0 from Table 2's initial values."""
    theta = np.zeros(PARAM_COUNT)
    p = unpack(theta)                    # views into theta
    for pre, n_in in (("r", N_FEAT_RHO), ("a", N_FEAT_ALPHA)):
        p[pre + "W1"][...] = rng.uniform(-1, 1, (n_in, HIDDEN)) / np.sqrt(n_in)
        p[pre + "b1"][...] = rng.uniform(-1, 1, HIDDEN) / np.sqrt(n_in)
        p[pre + "W2"][...] = rng.uniform(-1, 1, (HIDDEN, HIDDEN)) / np.sqrt(HIDDEN)
        p[pre + "b2"][...] = rng.uniform(-1, 1, HIDDEN) / np.sqrt(HIDDEN)
        if head_scale > 0:
            p[pre + "w3"][...] = rng.uniform(-head_scale, head_scale, HIDDEN)
            p[pre + "b3"][...] = rng.uniform(-head_scale, head_scale)
    p["l_rho0"][...] = logit_of_rho(np.asarray(TABLE2_RHO0))
    p["l_alpha0"][...] = logit_of_alpha(TABLE2_ALPHA0)
    return theta


def row_kinds(inst) -> np.ndarray:
    """Cone-kind index (0 zero, 1 nonnegative, 2 SOC, 3 PSD) of every row."""
    out = []
    for c in inst.cones:
        n = c.size * (c.size + 1) // 2 if c.kind == "psd" else c.size
        out += [KINDS.index(c.kind)] * n
    return np.asarray(out, np.int64)


class _Data:
    """The instance as float64 CPU tensors (dense: the oracle runs small
    instances)."""

    def __init__(self, inst):
        self.A = torch.from_numpy(inst.A.toarray().astype(np.float64))
        self.P = torch.from_numpy(inst.P.toarray().astype(np.float64))
        self.q = torch.from_numpy(np.asarray(inst.q, np.float64))
        self.b = torch.from_numpy(np.asarray(inst.b, np.float64))


def _inf(v):
    return v.abs().max() if v.numel() else v.new_zeros(())


def _normalised(r, N):
    # a zero normaliser means r = 0 as well: rbar = 0, no gradient through N
    return r / N if float(N.detach()) > 0.0 else torch.zeros_like(r)


def _mlp(xi, p, pre):
    h1 = torch.relu(xi @ p[pre + "W1"] + p[pre + "b1"])
    h2 = torch.relu(h1 @ p[pre + "W2"] + p[pre + "b2"])
    return h2 @ p[pre + "w3"] + p[pre + "b3"]


def squash_rho(l):
    return torch.exp((np.log(RHO_MAX) - np.log(RHO_MIN)) * torch.sigmoid(l) + np.log(RHO_MIN))


def squash_alpha(l):
    return 2.0 * torch.sigmoid(l)


def kkt(d: _Data, x, s, y):
    """(r_p, r_d, N_p, N_d) at z = (x, s, y) (App. E; r_d per reading R2)."""
    Ax, Aty, Px = d.A @ x, d.A.T @ y, d.P @ x
    rp = Ax + s - d.b
    rd = Px + d.q - Aty
    Np = torch.stack([_inf(Ax), _inf(s), _inf(d.b)]).max()
    Nd = torch.stack([_inf(Px), _inf(d.q), _inf(Aty)]).max()
    return rp, rd, Np, Nd


def policy_step(d: _Data, p, l_rho, l_alpha, x, s, y, s_prev=None, st_prev=None):
    """One policy evaluation at z^k: (l_rho^{k+1}, l_alpha^{k+1}, rho^k,
    alpha^k) from l^k and the features; s_prev = s^{k-1} and st_prev = the
    s~ that produced s^k, both None at k = 0 (the ADMM residuals are then 0)."""
    rp, rd, Np, Nd = kkt(d, x, s, y)
    rbp, rbd = _normalised(rp, Np), _normalised(rd, Nd)
    zero = torch.zeros_like(s)
    dp = zero if st_prev is None else s - st_prev
    dd = zero if s_prev is None else s - s_prev
    gd = torch.log(_inf(rbd) + EPS)
    gp = torch.log(_inf(rbp) + EPS)
    gdp = torch.log(_inf(dp) + EPS)
    gdd = torch.log(_inf(dd) + EPS)
    xi_r = torch.stack([l_rho, s, y, rbp, gd.expand_as(s), dp, dd], dim=1)
    xi_a = torch.stack([l_alpha, gp, gd, gdp, gdd])
    l_rho1 = l_rho + _mlp(xi_r, p, "r")
    l_alpha1 = l_alpha + _mlp(xi_a, p, "a")
    return l_rho1, l_alpha1, squash_rho(l_rho1), squash_alpha(l_alpha1)


def _loss_term(d: _Data, x, s, y, Dd, Dp):
    rp, rd, _, _ = kkt(d, x, s, y)
    return torch.log((rd @ rd) / Dd + (rp @ rp) / Dp)


def _t(a, grad=False):
    return torch.tensor(np.asarray(a, np.float64), requires_grad=grad)


def unroll_policy_forward(inst, theta, K: int, x0=None, s0=None, y0=None, sigma: float = 1e-6,
                          denominators=None) -> dict:
    """K steps with the policy choosing (rho^k, alpha^k) at every iterate;
    z^0 = 0 unless given.  Returns the tape (each step's COSMO intermediates
    and the policy's inputs), rho [K, m], alpha [K], the loss, and z^K.
    denominators: (|r_d^0|^2, |r_p^0|^2) to use instead of z^0's (the loss
    holds them constant; finite differences in z^0 need them fixed)."""
    n, m = inst.A.shape[1], inst.A.shape[0]
    d = _Data(inst)
    p = unpack(torch.from_numpy(np.asarray(theta, np.float64)))
    x = np.zeros(n) if x0 is None else np.asarray(x0, np.float64).copy()
    s = np.zeros(m) if s0 is None else np.asarray(s0, np.float64).copy()
    y = np.zeros(m) if y0 is None else np.asarray(y0, np.float64).copy()
    l_rho = p["l_rho0"][torch.from_numpy(row_kinds(inst))].clone()
    l_alpha = p["l_alpha0"].clone()
    if denominators is None:
        with torch.no_grad():
            rp0, rd0, _, _ = kkt(d, _t(x), _t(s), _t(y))
        Dd, Dp = float(rd0 @ rd0) or 1.0, float(rp0 @ rp0) or 1.0
    else:
        Dd, Dp = denominators
    tape, rhos, alphas, loss = [], np.zeros((K, m)), np.zeros(K), 0.0
    s_prev = st_prev = None
    for k in range(K):
        with torch.no_grad():
            l_rho1, l_alpha1, rho, alpha = policy_step(d, p, l_rho, l_alpha, _t(x), _t(s), _t(y),
                                                       None if s_prev is None else _t(s_prev),
                                                       None if st_prev is None else _t(st_prev))
        rhos[k], alphas[k] = rho.numpy(), float(alpha)
        st = step_forward(inst, x, s, y, rhos[k], alphas[k], sigma)
        tape.append(dict(step=st, l_rho=l_rho.numpy().copy(), l_alpha=float(l_alpha),
                         s_prev=s_prev, st_prev=st_prev))
        s_prev, st_prev = s, st["st"]
        x, s, y = st["xn"], st["sn"], st["yn"]
        l_rho, l_alpha = l_rho1, l_alpha1
        with torch.no_grad():
            loss += float(_loss_term(d, _t(x), _t(s), _t(y), Dd, Dp))
    return dict(tape=tape, rho=rhos, alpha=alphas, loss=loss, x=x, s=s, y=y, Dd=Dd, Dp=Dp,
                l_rho=l_rho.numpy(), l_alpha=float(l_alpha))


def unroll_policy_backward(inst, theta, fw: dict, sigma: float = 1e-6):
    """Gradient of the loss with respect to the policy parameters (flat, like
    theta, l^0 included) and to z^0; also the cotangents of rho^k and
    alpha^k that the unroll delivers (grho [K, m], galpha [K])."""
    K = len(fw["tape"])
    m = inst.A.shape[0]
    d = _Data(inst)
    theta_t = _t(theta, grad=True)
    p = unpack(theta_t)
    Dd, Dp = fw["Dd"], fw["Dp"]

    def loss_grad(x, s, y):
        xs = [_t(v, grad=True) for v in (x, s, y)]
        return [g.numpy() for g in torch.autograd.grad(_loss_term(d, *xs, Dd, Dp), xs)]

    gx, gs, gy = loss_grad(fw["x"], fw["s"], fw["y"])
    C_rho, C_alpha = np.zeros(m), 0.0          # cotangents of l^{k+1}
    pend_s = pend_st = None
    g_theta = np.zeros_like(np.asarray(theta, np.float64))
    grho, galpha = np.zeros((K, m)), np.zeros(K)
    for k in range(K - 1, -1, -1):
        rec = fw["tape"][k]
        st = rec["step"]
        gx, gs, gy, grho[k], galpha[k] = step_backward(inst, st, gx, gs, gy, sigma, gst_extra=pend_st)
        if pend_s is not None:
            gs = gs + pend_s
        if k >= 1:
            lx, ls, ly = loss_grad(st["x"], st["s"], st["y"])
            gx, gs, gy = gx + lx, gs + ls, gy + ly
        ins = [_t(rec["l_rho"], True), _t(rec["l_alpha"], True), _t(st["x"], True), _t(st["s"], True),
               _t(st["y"], True)]
        prev = [] if k == 0 else [_t(rec["s_prev"], True), _t(rec["st_prev"], True)]
        l_rho1, l_alpha1, rho, alpha = policy_step(d, p, *ins, *prev)
        outs = torch.autograd.grad([rho, alpha, l_rho1, l_alpha1], [theta_t] + ins + prev,
                                   grad_outputs=[_t(grho[k]), _t(galpha[k]), _t(C_rho), _t(C_alpha)],
                                   allow_unused=True)
        outs = [np.zeros(1) if o is None else o.numpy() for o in outs]
        g_theta += outs[0]
        C_rho, C_alpha = outs[1], float(outs[2])
        gx, gs, gy = gx + outs[3], gs + outs[4], gy + outs[5]
        pend_s, pend_st = (outs[6], outs[7]) if k >= 1 else (None, None)
    # l^0 is the per-kind logit broadcast over the rows
    off = PARAM_COUNT - len(KINDS) - 1
    g_theta[off:off + len(KINDS)] += np.bincount(row_kinds(inst), weights=C_rho, minlength=len(KINDS))
    g_theta[PARAM_COUNT - 1] += C_alpha
    return dict(g_theta=g_theta, gx0=gx, gs0=gs, gy0=gy, grho=grho, galpha=galpha)


def log_residual_loss(inst, zs) -> float:
    """The loss over a given trajectory zs = [z^0, ..., z^K] (z = (x, s, y))."""
    d = _Data(inst)
    with torch.no_grad():
        rp0, rd0, _, _ = kkt(d, *(_t(v) for v in zs[0]))
        Dd, Dp = float(rd0 @ rd0) or 1.0, float(rp0 @ rp0) or 1.0
        return float(sum(_loss_term(d, *(_t(v) for v in z), Dd, Dp) for z in zs[1:]))
