"""Python binding of the C ABI: stacks a list of conic instances into one
super-batch (device tensors owned by PyTorch), creates the plan, and exposes
the forward / backward / loss / projection calls plus a
torch.autograd.Function wrapper.  Marshalling only: no step of the method is
computed here.

An instance is any object with attributes P (n x n scipy sparse, symmetric),
q [n], A (m x n scipy sparse), b [m] and cones (objects with .kind in
{"zero", "nonneg", "soc", "psd"} and .size = rows, or matrix order for psd).
An instance may describe a dense sub-block of A in meta["dense"] =
{"col0", "rows", "cols", "place": [(row0, scale), ...]} (first scale 1): the
library then receives that block once as a dense array (cosmo_dense_block)
and A without those entries as CSR.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_TORCH_DT = {L.COSMO_F32: torch.float32, L.COSMO_F64: torch.float64}
_NP_DT = {L.COSMO_F32: np.float32, L.COSMO_F64: np.float64}


def _dt_code(dtype) -> int:
    if dtype in (torch.float32, np.float32, "f32", "float32"):
        return L.COSMO_F32
    if dtype in (torch.float64, np.float64, "f64", "float64"):
        return L.COSMO_F64
    raise ValueError(f"unsupported dtype {dtype}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _psd_rows(p: int) -> int:
    return p * (p + 1) // 2


def _split_dense(inst, npdt):
    """(CSR remainder of A, dense block G or None, its description).  G is
    read from A at the first placement (scale 1); every other placement
    must hold exactly scale * G in the run dtype, and the entries of every
    placement are dropped from the CSR remainder.  A copy, no arithmetic."""
    desc = (getattr(inst, "meta", None) or {}).get("dense")
    A = inst.A.tocsr()
    if not desc:
        return A, None, None
    r0, c0 = int(desc["place"][0][0]), int(desc["col0"])
    rows, cols = int(desc["rows"]), int(desc["cols"])
    if float(desc["place"][0][1]) != 1.0:
        raise ValueError("the first placement of a dense block must have scale 1")
    G = A[r0:r0 + rows, c0:c0 + cols].toarray().astype(npdt)
    for (row0, sc) in desc["place"][1:]:
        blk = A[int(row0):int(row0) + rows, c0:c0 + cols].toarray().astype(npdt)
        if not np.array_equal(blk, (npdt(sc) * G).astype(npdt)):
            raise ValueError("a dense placement does not hold scale * G")
    C = A.tocoo()
    keep = np.ones(C.nnz, bool)
    for (row0, _) in desc["place"]:
        keep &= ~((C.row >= int(row0)) & (C.row < int(row0) + rows) & (C.col >= c0) & (C.col < c0 + cols))
    import scipy.sparse as sp
    R = sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=A.shape)
    return R, G, desc


@dataclass
class ForwardResult:
    x: torch.Tensor
    s: torch.Tensor
    y: torch.Tensor
    tape: Optional[torch.Tensor]


@dataclass
class PolicyForwardResult:
    x: torch.Tensor
    s: torch.Tensor
    y: torch.Tensor
    rho: torch.Tensor
    alpha: torch.Tensor
    loss: torch.Tensor
    tape: Optional[torch.Tensor]
    ptape: torch.Tensor
    pws: torch.Tensor


@dataclass
class BackwardResult:
    grho: torch.Tensor
    galpha: torch.Tensor
    gx0: torch.Tensor
    gs0: torch.Tensor
    gy0: torch.Tensor


class CosmoBatch:
    """A super-batch of B instances on one GPU and its plan (App. C,
    "super-batches").  Hyperparameters: rho [K, m_tot] per row, alpha [K, B]."""

    def __init__(self, instances: Sequence, *, K: int, dtype=torch.float32, sigma: float = 1e-6,
                 cg_tol: Optional[float] = None, cg_max_iter: int = 500, eig_max_sweeps: int = 60,
                 eig_tol: float = 0.0, eig_refine: int = 1, eig_warm_start: bool = True, dense: bool = True,
                 dense_f32: bool = False, device="cuda:0"):
        self.device = torch.device(device)
        self.code = _dt_code(dtype)
        self.dtype = _TORCH_DT[self.code]
        npdt = _NP_DT[self.code]
        self.K, self.B = int(K), len(instances)
        if cg_tol is None:
            # the paper's CG relative tolerance (1e-8, standalone-results table
            # caption); float64 runs tighten it for float64 parity
            cg_tol = 1e-8 if self.code == L.COSMO_F32 else 1e-12
        ns = [int(inst.A.shape[1]) for inst in instances]
        ms = [int(inst.A.shape[0]) for inst in instances]
        self.n_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
        self.m_off = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
        self.n_tot, self.m_tot = int(self.n_off[-1]), int(self.m_off[-1])
        # stacked CSR of A and P (block diagonal), built per instance
        arp, acol, aval, prp, pcol, pval = [np.zeros(1, np.int64)], [], [], [np.zeros(1, np.int64)], [], []
        annz = pnnz = 0
        kinds, sizes = [], []
        dense_parts = []   # (instance, G, description)
        for i, inst in enumerate(instances):
            if dense:
                A, G, desc = _split_dense(inst, npdt)
                if G is not None:
                    dense_parts.append((i, G, desc))
            else:
                A = inst.A.tocsr()
            A.sort_indices()
            arp.append(A.indptr[1:].astype(np.int64) + annz)
            acol.append(A.indices.astype(np.int32) + np.int32(self.n_off[i]))
            aval.append(A.data.astype(npdt))
            annz += A.nnz
            Pm = inst.P.tocsr()
            Pm.sort_indices()
            prp.append(Pm.indptr[1:].astype(np.int64) + pnnz)
            pcol.append(Pm.indices.astype(np.int32) + np.int32(self.n_off[i]))
            pval.append(Pm.data.astype(npdt))
            pnnz += Pm.nnz
            for c in inst.cones:
                kinds.append(L.CONE_CODES[c.kind])
                sizes.append(int(c.size))
        dev = self.device
        self.A_rowptr = torch.from_numpy(np.concatenate(arp)).to(dev)
        self.A_col = torch.from_numpy(np.concatenate(acol) if acol else np.zeros(0, np.int32)).to(dev)
        self.A_val = torch.from_numpy(np.concatenate(aval)).to(dev)
        self.A_nnz = annz
        self.P_nnz = pnnz
        if pnnz:
            self.P_rowptr = torch.from_numpy(np.concatenate(prp)).to(dev)
            self.P_col = torch.from_numpy(np.concatenate(pcol)).to(dev)
            self.P_val = torch.from_numpy(np.concatenate(pval)).to(dev)
        else:
            self.P_rowptr = self.P_col = self.P_val = None
        self.q = torch.from_numpy(np.concatenate([np.asarray(inst.q, np.float64) for inst in instances]).astype(npdt)).to(dev)
        self.b = torch.from_numpy(np.concatenate([np.asarray(inst.b, np.float64) for inst in instances]).astype(npdt)).to(dev)
        self.cone_kind = np.asarray(kinds, np.int32)
        self.cone_size = np.asarray(sizes, np.int32)
        # dense blocks: one device array, each block row-major with ld a
        # multiple of 16 bytes (every block starts 16-byte aligned)
        # dense_f32: a float64 batch stores its dense blocks as float32; only
        # blocks whose values are float32 numbers qualify (then nothing is lost)
        gdt = np.float32 if dense_f32 else npdt
        if dense_f32:
            for _, G, _ in dense_parts:
                if not np.array_equal(G.astype(np.float32).astype(G.dtype), G):
                    raise ValueError("dense_f32: a dense block has values that are not float32 numbers")
        ve = 16 // np.dtype(gdt).itemsize
        self.n_dense = len(dense_parts)
        self._dense_desc = (L.CosmoDenseBlock * max(1, self.n_dense))()
        self.dense_val = None
        if dense_parts:
            chunks, offs, off = [], [], 0
            for k, (i, G, desc) in enumerate(dense_parts):
                rows, cols = G.shape
                ld = (cols + ve - 1) // ve * ve
                Gp = np.zeros((rows, ld), gdt)
                Gp[:, :cols] = G
                chunks.append(Gp.ravel())
                d = self._dense_desc[k]
                d.rows, d.cols, d.ld = rows, cols, ld
                d.col0 = int(self.n_off[i]) + int(desc["col0"])
                d.n_place = len(desc["place"])
                d.val_f32 = 1 if gdt == np.float32 else 0
                for q, (row0, sc) in enumerate(desc["place"]):
                    d.row0[q] = int(self.m_off[i]) + int(row0)
                    d.scale[q] = float(sc)
                offs.append(off)   # element offset in the device array
                off += Gp.size
            self.dense_val = torch.from_numpy(np.concatenate(chunks)).to(self.device)
            base = self.dense_val.data_ptr()
            for k in range(self.n_dense):
                self._dense_desc[k].val = base + offs[k] * np.dtype(gdt).itemsize
        self.instances_meta = [(ns[i], ms[i]) for i in range(self.B)]
        prob = L.CosmoProblem()
        prob.B = self.B
        prob.n_off = self.n_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        prob.m_off = self.m_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        prob.A_rowptr = self.A_rowptr.data_ptr()
        prob.A_col = self.A_col.data_ptr()
        prob.A_val = self.A_val.data_ptr()
        prob.A_nnz = annz
        prob.P_rowptr = self.P_rowptr.data_ptr() if pnnz else None
        prob.P_col = self.P_col.data_ptr() if pnnz else None
        prob.P_val = self.P_val.data_ptr() if pnnz else None
        prob.P_nnz = pnnz
        prob.q = self.q.data_ptr()
        prob.b = self.b.data_ptr()
        prob.n_cones = len(kinds)
        prob.cone_kind = self.cone_kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        prob.cone_size = self.cone_size.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        prob.n_dense = self.n_dense
        prob.dense = ctypes.cast(self._dense_desc, ctypes.POINTER(L.CosmoDenseBlock))
        opt = L.CosmoOptions()
        opt.dtype = self.code
        opt.K = self.K
        opt.sigma = float(sigma)
        opt.cg_tol = float(cg_tol)
        opt.cg_max_iter = int(cg_max_iter)
        opt.eig_max_sweeps = int(eig_max_sweeps)
        opt.eig_tol = float(eig_tol)
        opt.eig_refine = int(eig_refine)
        opt.eig_warm_start = int(bool(eig_warm_start))
        self.opt = opt
        lib = L.lib()
        torch.cuda.synchronize(dev)
        h = ctypes.c_void_p()
        L.check(lib.cosmo_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt)), "cosmo_plan_create")
        self._plan = h
        f, t, b = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        L.check(lib.cosmo_workspace_size(h, ctypes.byref(f), ctypes.byref(t), ctypes.byref(b)), "cosmo_workspace_size")
        self.fwd_ws_bytes, self.tape_bytes, self.bwd_ws_bytes = f.value, t.value, b.value
        self.esz = 4 if self.code == L.COSMO_F32 else 8

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "_plan", None):
            L.lib().cosmo_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ---------------------------------------------------------------
    def _buf(self, nbytes: int) -> torch.Tensor:
        return torch.empty((max(nbytes, self.esz) + self.esz - 1) // self.esz, dtype=self.dtype, device=self.device)

    def new_tape(self) -> torch.Tensor:
        return self._buf(self.tape_bytes)

    def new_fwd_ws(self) -> torch.Tensor:
        return self._buf(self.fwd_ws_bytes)

    def new_bwd_ws(self) -> torch.Tensor:
        return self._buf(self.bwd_ws_bytes)

    def new_stats(self) -> torch.Tensor:
        return torch.zeros((self.B, L.STATS_INTS), dtype=torch.int32, device=self.device)

    @staticmethod
    def stats_dict(stats: torch.Tensor):
        s = stats.cpu().numpy()
        return {k: s[:, i].copy() for i, k in enumerate(L.STATS_FIELDS)}

    def _check_vec(self, t, n, name):
        if t is None:
            return None
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: need a contiguous {self.dtype} tensor of {n} elements on {self.device}")
        return t

    # -- calls ---------------------------------------------------------------
    def forward(self, rho: torch.Tensor, alpha: torch.Tensor, x0=None, s0=None, y0=None, *, tape=True,
                stats: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                out: Optional[tuple] = None) -> ForwardResult:
        self._check_vec(rho, self.K * self.m_tot, "rho")
        self._check_vec(alpha, self.K * self.B, "alpha")
        for t, n, nm in ((x0, self.n_tot, "x0"), (s0, self.m_tot, "s0"), (y0, self.m_tot, "y0")):
            self._check_vec(t, n, nm)
        if isinstance(tape, torch.Tensor):
            tp = tape
        else:
            tp = self.new_tape() if tape else None
        ws = ws if ws is not None else self.new_fwd_ws()
        if out is None:
            out = (torch.empty(self.n_tot, dtype=self.dtype, device=self.device),
                   torch.empty(self.m_tot, dtype=self.dtype, device=self.device),
                   torch.empty(self.m_tot, dtype=self.dtype, device=self.device))
        x, s, y = out
        st = L.lib().cosmo_unroll_forward(self._plan, _ptr(rho), _ptr(alpha), _ptr(x0), _ptr(s0), _ptr(y0),
                                          _ptr(x), _ptr(s), _ptr(y), _ptr(tp), _ptr(ws), _ptr(stats),
                                          _stream(self.device))
        L.check(st, "cosmo_unroll_forward")
        return ForwardResult(x, s, y, tp)

    def backward(self, rho, alpha, tape, gx=None, gs=None, gy=None, *, stats=None, ws=None,
                 out: Optional[tuple] = None) -> BackwardResult:
        if tape is None:
            raise ValueError("backward needs the tape of a forward call")
        for t, n, nm in ((gx, self.n_tot, "gx"), (gs, self.m_tot, "gs"), (gy, self.m_tot, "gy")):
            self._check_vec(t, n, nm)
        ws = ws if ws is not None else self.new_bwd_ws()
        if out is None:
            out = (torch.empty((self.K, self.m_tot), dtype=self.dtype, device=self.device),
                   torch.empty((self.K, self.B), dtype=self.dtype, device=self.device),
                   torch.empty(self.n_tot, dtype=self.dtype, device=self.device),
                   torch.empty(self.m_tot, dtype=self.dtype, device=self.device),
                   torch.empty(self.m_tot, dtype=self.dtype, device=self.device))
        grho, galpha, gx0, gs0, gy0 = out
        st = L.lib().cosmo_unroll_backward(self._plan, _ptr(rho), _ptr(alpha), _ptr(tape), _ptr(gx), _ptr(gs),
                                           _ptr(gy), _ptr(grho), _ptr(galpha), _ptr(gx0), _ptr(gs0), _ptr(gy0),
                                           _ptr(ws), _ptr(stats), _stream(self.device))
        L.check(st, "cosmo_unroll_backward")
        return BackwardResult(grho, galpha, gx0, gs0, gy0)

    # -- vanilla COSMO to tolerance (cosmo_solve) ---------------------------------
    def solve(self, *, rho0: float = 0.1, eq_scale: float = 1e3, alpha: float = 1.6, eps_abs: float = 1e-3,
              eps_rel: float = 1e-3, max_iter: int = 10000, interval: int = 40, tol_factor: float = 5.0,
              rho_min: float = 1e-6, rho_max: float = 1e6, adapt: bool = True, x0=None, s0=None, y0=None,
              stats=None, ws=None):
        """COSMO run to tolerance with the residual-balancing penalty, checked
        every K steps (K = 1: exact counts).  Returns (iters [B] numpy int32,
        -1 where max_iter came first; final penalty scalars [B]; x, s, y, each
        instance's slice the iterate at its own count)."""
        opt = L.CosmoSolveOptions(rho0=rho0, eq_scale=eq_scale, alpha=alpha, eps_abs=eps_abs, eps_rel=eps_rel,
                                  tol_factor=tol_factor, rho_min=rho_min, rho_max=rho_max, max_iter=max_iter,
                                  interval=interval, adapt=int(adapt), pad=0)
        z = []
        for t, n in ((x0, self.n_tot), (s0, self.m_tot), (y0, self.m_tot)):
            z.append(torch.zeros(n, dtype=self.dtype, device=self.device) if t is None else t.clone())
        x, s, y = z
        sb = ctypes.c_size_t()
        L.check(L.lib().cosmo_solve_size(self._plan, ctypes.byref(sb)), "cosmo_solve_size")
        sws = torch.empty(max(sb.value, 1), dtype=torch.uint8, device=self.device)
        ws = ws if ws is not None else self.new_fwd_ws()
        iters = np.zeros(self.B, np.int32)
        rho = np.zeros(self.B, np.float64)
        st = L.lib().cosmo_solve(self._plan, ctypes.byref(opt), _ptr(x), _ptr(s), _ptr(y),
                                 iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(ws), _ptr(sws),
                                 _ptr(stats), _stream(self.device))
        L.check(st, "cosmo_solve")
        return iters, rho, x, s, y

    # -- learned policy (cosmo_policy_forward / cosmo_policy_backward) -----------
    def policy_sizes(self):
        """(ptape_bytes, pws_bytes) of the policy calls."""
        pt, pw = ctypes.c_size_t(), ctypes.c_size_t()
        L.check(L.lib().cosmo_policy_sizes(self._plan, ctypes.byref(pt), ctypes.byref(pw)), "cosmo_policy_sizes")
        return pt.value, pw.value

    def policy_forward(self, theta: torch.Tensor, x0=None, s0=None, y0=None, *, tape=True, ptape=None, pws=None,
                       ws=None, stats=None) -> "PolicyForwardResult":
        """K steps with the policy choosing rho^k and alpha^k; returns the final
        iterate, the chosen rho [K, m_tot] and alpha [K, B], the per-instance
        log-residual loss and the buffers the backward pass needs."""
        self._check_vec(theta, L.COSMO_POLICY_PARAMS, "theta")
        for t, n, nm in ((x0, self.n_tot, "x0"), (s0, self.m_tot, "s0"), (y0, self.m_tot, "y0")):
            self._check_vec(t, n, nm)
        pt_bytes, pw_bytes = self.policy_sizes()
        tp = tape if isinstance(tape, torch.Tensor) else (self.new_tape() if tape else None)
        ptape = ptape if ptape is not None else torch.empty(pt_bytes, dtype=torch.uint8, device=self.device)
        pws = pws if pws is not None else torch.empty(pw_bytes, dtype=torch.uint8, device=self.device)
        ws = ws if ws is not None else self.new_fwd_ws()
        rho = torch.empty((self.K, self.m_tot), dtype=self.dtype, device=self.device)
        alpha = torch.empty((self.K, self.B), dtype=self.dtype, device=self.device)
        x = torch.empty(self.n_tot, dtype=self.dtype, device=self.device)
        s = torch.empty(self.m_tot, dtype=self.dtype, device=self.device)
        y = torch.empty(self.m_tot, dtype=self.dtype, device=self.device)
        loss = torch.empty(self.B, dtype=self.dtype, device=self.device)
        st = L.lib().cosmo_policy_forward(self._plan, _ptr(theta), _ptr(x0), _ptr(s0), _ptr(y0), _ptr(rho),
                                          _ptr(alpha), _ptr(x), _ptr(s), _ptr(y), _ptr(loss), _ptr(tp), _ptr(ptape),
                                          _ptr(ws), _ptr(pws), _ptr(stats), _stream(self.device))
        L.check(st, "cosmo_policy_forward")
        return PolicyForwardResult(x, s, y, rho, alpha, loss, tp, ptape, pws)

    def policy_backward(self, theta: torch.Tensor, fw: "PolicyForwardResult", *, ws=None, stats=None):
        """(gtheta, grho [K, m_tot], galpha [K, B], gx0, gs0, gy0) of the summed loss."""
        if fw.tape is None:
            raise ValueError("policy_backward needs a forward run with a tape")
        self._check_vec(theta, L.COSMO_POLICY_PARAMS, "theta")
        ws = ws if ws is not None else self.new_bwd_ws()
        gtheta = torch.empty(L.COSMO_POLICY_PARAMS, dtype=self.dtype, device=self.device)
        grho = torch.empty((self.K, self.m_tot), dtype=self.dtype, device=self.device)
        galpha = torch.empty((self.K, self.B), dtype=self.dtype, device=self.device)
        gx0 = torch.empty(self.n_tot, dtype=self.dtype, device=self.device)
        gs0 = torch.empty(self.m_tot, dtype=self.dtype, device=self.device)
        gy0 = torch.empty(self.m_tot, dtype=self.dtype, device=self.device)
        st = L.lib().cosmo_policy_backward(self._plan, _ptr(theta), _ptr(fw.rho), _ptr(fw.alpha), _ptr(fw.tape),
                                           _ptr(fw.ptape), _ptr(gtheta), _ptr(grho), _ptr(galpha), _ptr(gx0),
                                           _ptr(gs0), _ptr(gy0), _ptr(ws), _ptr(fw.pws), _ptr(stats),
                                           _stream(self.device))
        L.check(st, "cosmo_policy_backward")
        return gtheta, grho, galpha, gx0, gs0, gy0

    def residual_loss(self, x, s, y, *, grad=True, ws=None):
        ws = ws if ws is not None else self.new_fwd_ws()
        loss = torch.empty(self.B, dtype=self.dtype, device=self.device)
        g = (torch.empty(self.n_tot, dtype=self.dtype, device=self.device),
             torch.empty(self.m_tot, dtype=self.dtype, device=self.device),
             torch.empty(self.m_tot, dtype=self.dtype, device=self.device)) if grad else (None, None, None)
        st = L.lib().cosmo_residual_loss(self._plan, _ptr(x), _ptr(s), _ptr(y), _ptr(loss), _ptr(g[0]),
                                         _ptr(g[1]), _ptr(g[2]), _ptr(ws), _stream(self.device))
        L.check(st, "cosmo_residual_loss")
        return loss, g

    def tape_iterate(self, tape: torch.Tensor, k: int):
        """Views of (x^k, s^k, y^k) and, for k < K, (x~, s~) of step k."""
        offs = [ctypes.c_size_t() for _ in range(5)]
        want_step = k < self.K
        args = [ctypes.byref(o) for o in offs[:3]] + ([ctypes.byref(o) for o in offs[3:]] if want_step else [None, None])
        L.check(L.lib().cosmo_tape_offsets(self._plan, int(k), *args), "cosmo_tape_offsets")
        e = self.esz
        n, m = self.n_tot, self.m_tot
        x = tape[offs[0].value // e: offs[0].value // e + n]
        s = tape[offs[1].value // e: offs[1].value // e + m]
        y = tape[offs[2].value // e: offs[2].value // e + m]
        if not want_step:
            return x, s, y, None, None
        return (x, s, y, tape[offs[3].value // e: offs[3].value // e + n],
                tape[offs[4].value // e: offs[4].value // e + m])

    def split_n(self, v):
        return [v[self.n_off[i]:self.n_off[i + 1]] for i in range(self.B)]

    def split_m(self, v):
        return [v[..., self.m_off[i]:self.m_off[i + 1]] for i in range(self.B)]

    # -- measurement -------------------------------------------------------------
    def set_tap(self, tap: Optional[torch.Tensor]):
        """Per-step taps of the backward (cosmo_plan_set_tap): tap [K, 2, m_tot]
        of the batch's dtype receives v^k and the cotangent of the projection's
        output, every row, at every step; None stops."""
        if tap is not None:
            if tap.dtype != self.dtype or tap.device != self.device or not tap.is_contiguous() or \
                    tuple(tap.shape) != (self.K, 2, self.m_tot):
                raise ValueError(f"tap must be a contiguous {self.dtype} tensor of shape ({self.K}, 2, {self.m_tot})")
        self._tap = tap
        L.check(L.lib().cosmo_plan_set_tap(self._plan, _ptr(tap)), "cosmo_plan_set_tap")

    def set_profiling(self, on: bool):
        L.check(L.lib().cosmo_plan_set_profiling(self._plan, int(on)), "cosmo_plan_set_profiling")

    # -- schedules ----------------------------------------------------------------
    def set_pcg_form(self, form: int):
        """CG schedule: 0 one workgroup per instance, 1..4 cooperative (that
        many workgroups per compute unit at most)."""
        L.check(L.lib().cosmo_plan_set_pcg_form(self._plan, int(form)), "cosmo_plan_set_pcg_form")

    def pcg_form(self) -> int:
        f = ctypes.c_int32()
        L.check(L.lib().cosmo_plan_get_pcg_form(self._plan, ctypes.byref(f)), "cosmo_plan_get_pcg_form")
        return f.value

    def set_graph(self, enable: bool):
        """Graph mode: forward and backward calls record their launch
        sequence once per set of buffers and replay it afterwards."""
        L.check(L.lib().cosmo_plan_set_graph(self._plan, int(bool(enable))), "cosmo_plan_set_graph")

    def graph(self) -> bool:
        f = ctypes.c_int32()
        L.check(L.lib().cosmo_plan_get_graph(self._plan, ctypes.byref(f)), "cosmo_plan_get_graph")
        return bool(f.value)

    def set_psd_schedule(self, eig_threads, vjp_threads: int = 1024):
        """PSD launch shapes: eigensolve threads per order class (p <= 32,
        <= 64, <= 128, larger; defaults 64, 256, 512, 1024, alternatives
        twice that for the first three) and DK VJP threads (1024 or 512)."""
        arr = (ctypes.c_int32 * 4)(*[int(t) for t in eig_threads])
        L.check(L.lib().cosmo_plan_set_psd_schedule(self._plan, arr, int(vjp_threads)), "cosmo_plan_set_psd_schedule")

    def psd_schedule(self):
        """(eigensolve threads per order class, DK VJP threads) in use."""
        arr, v = (ctypes.c_int32 * 4)(), ctypes.c_int32()
        L.check(L.lib().cosmo_plan_get_psd_schedule(self._plan, arr, ctypes.byref(v)), "cosmo_plan_get_psd_schedule")
        return [int(t) for t in arr], int(v.value)

    def psd_tune_ms(self):
        """The last autotune's PSD timings: {"default"|"alt": [class 0..3
        eigensolve ms over one forward, DK VJP ms]}, -1 where not timed."""
        ms = (ctypes.c_double * 10)()
        L.check(L.lib().cosmo_plan_psd_tune_ms(self._plan, ms), "cosmo_plan_psd_tune_ms")
        return {"default": [float(x) for x in ms[:5]], "alt": [float(x) for x in ms[5:]]}

    def schedule(self) -> dict:
        """The plan's whole launch schedule (CG form, graph mode, PSD shapes)."""
        sc = L.CosmoSchedule()
        L.check(L.lib().cosmo_plan_get_schedule(self._plan, ctypes.byref(sc)), "cosmo_plan_get_schedule")
        return sc.as_dict()

    def set_schedule(self, pcg_form: int, graph: bool, eig_threads, vjp_threads: int):
        sc = L.CosmoSchedule(int(pcg_form), int(bool(graph)), (ctypes.c_int32 * 4)(*[int(t) for t in eig_threads]),
                             int(vjp_threads))
        L.check(L.lib().cosmo_plan_set_schedule(self._plan, ctypes.byref(sc)), "cosmo_plan_set_schedule")

    def signature(self) -> str:
        """Key of this plan's entry in a schedule cache."""
        buf = ctypes.create_string_buffer(256)
        L.check(L.lib().cosmo_plan_signature(self._plan, buf, 256), "cosmo_plan_signature")
        return buf.value.decode()

    def autotune_cached(self, rho: torch.Tensor, alpha: torch.Tensor, path: str,
                        ws: Optional[torch.Tensor] = None) -> bool:
        """Schedule from the cache file at `path` when it holds this plan's
        signature (returns True), else autotune and record it (False)."""
        rho = self._check_vec(rho.contiguous(), self.K * self.m_tot, "rho")
        alpha = self._check_vec(alpha.contiguous(), self.K * self.B, "alpha")
        ws = ws if ws is not None else self.new_fwd_ws()
        hit = ctypes.c_int32()
        L.check(L.lib().cosmo_plan_autotune_cached(self._plan, _ptr(rho), _ptr(alpha), _ptr(ws), _stream(self.device),
                                                    os.fsencode(path), ctypes.byref(hit)), "cosmo_plan_autotune_cached")
        return bool(hit.value)

    def autotune(self, rho: torch.Tensor, alpha: torch.Tensor, ws: Optional[torch.Tensor] = None):
        """Time the schedules (CG forms 0, 2, 4 eager; form 0 from a graph) on
        a forward unroll and keep the fastest; then the PSD launch shapes
        (psd_schedule(), psd_tune_ms()).  Returns (chosen CG form, [ms per
        schedule], -1 where not run).  graph() tells whether graph mode was
        chosen."""
        rho = self._check_vec(rho.contiguous(), self.K * self.m_tot, "rho")
        alpha = self._check_vec(alpha.contiguous(), self.K * self.B, "alpha")
        ws = ws if ws is not None else self.new_fwd_ws()
        ms = (ctypes.c_double * 4)()
        L.check(L.lib().cosmo_plan_autotune(self._plan, _ptr(rho), _ptr(alpha), _ptr(ws), _stream(self.device), ms),
                "cosmo_plan_autotune")
        return self.pcg_form(), [float(x) for x in ms]

    def profile_read(self, kind: int):
        n, ms = ctypes.c_int64(), ctypes.c_double()
        L.check(L.lib().cosmo_plan_profile_read(self._plan, int(kind), ctypes.byref(n), ctypes.byref(ms)),
                "cosmo_plan_profile_read")
        return n.value, ms.value


class CosmoUnroll(torch.autograd.Function):
    """(x^K, s^K, y^K) = K unrolled COSMO steps from (x^0, s^0, y^0) with
    per-step (rho^k, alpha^k); backward by the library's reverse pass."""

    @staticmethod
    def forward(ctx, batch: CosmoBatch, rho, alpha, x0=None, s0=None, y0=None):
        r = batch.forward(rho.contiguous(), alpha.contiguous(), x0, s0, y0, tape=True)
        ctx.batch = batch
        ctx.has0 = (x0 is not None, s0 is not None, y0 is not None)
        ctx.save_for_backward(rho, alpha, r.tape)
        return r.x, r.s, r.y

    @staticmethod
    def backward(ctx, gx, gs, gy):
        rho, alpha, tape = ctx.saved_tensors
        b: CosmoBatch = ctx.batch
        g = [None if t is None else t.contiguous() for t in (gx, gs, gy)]
        r = b.backward(rho.contiguous(), alpha.contiguous(), tape, *g)
        return (None, r.grho.view_as(rho), r.galpha.view_as(alpha),
                r.gx0 if ctx.has0[0] else None, r.gs0 if ctx.has0[1] else None, r.gy0 if ctx.has0[2] else None)


class ResidualLoss(torch.autograd.Function):
    """Sum over instances of ||Ax + s - b||^2 + ||Px + q - A'y||^2."""

    @staticmethod
    def forward(ctx, batch: CosmoBatch, x, s, y):
        loss, g = batch.residual_loss(x.contiguous(), s.contiguous(), y.contiguous(), grad=True)
        ctx.save_for_backward(*g)
        return loss.sum()

    @staticmethod
    def backward(ctx, go):
        gx, gs, gy = ctx.saved_tensors
        return None, gx * go, gs * go, gy * go


# ---- standalone projections --------------------------------------------------

def _proj_ws(nblk: int, sizes: np.ndarray, device) -> torch.Tensor:
    nb = L.lib().cosmo_proj_workspace_size(int(nblk), sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return torch.empty(int(nb), dtype=torch.uint8, device=device)


def psd_proj(x: torch.Tensor, orders: Sequence[int], offsets: Optional[Sequence[int]] = None, *,
             max_sweeps: int = 60, eig_tol: float = 0.0, refine: int = 1, want_eig: bool = True):
    """Project each svec block of x onto the PSD cone (eq:psd-proj).
    Returns (out, eigvals [sum p], eigvecs [sum p^2]) ."""
    orders = np.asarray(orders, np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum([_psd_rows(int(p)) for p in orders])[:-1]])
    offsets = np.asarray(offsets, np.int64)
    code = _dt_code(x.dtype)
    out = torch.empty_like(x)
    lam = torch.empty(int(orders.sum()), dtype=x.dtype, device=x.device) if want_eig else None
    U = torch.empty(int((orders.astype(np.int64) ** 2).sum()), dtype=x.dtype, device=x.device) if want_eig else None
    ws = _proj_ws(len(orders), orders, x.device)
    st = L.lib().psd_proj(len(orders), orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), code, _ptr(x.contiguous()),
                          _ptr(out), _ptr(lam), _ptr(U), int(max_sweeps), float(eig_tol), int(refine), _ptr(ws),
                          _stream(x.device))
    L.check(st, "psd_proj")
    return out, lam, U


def psd_proj_vjp(eigvals, eigvecs, gout: torch.Tensor, orders, offsets=None):
    """Daleckii-Krein VJP of psd_proj (eq:psd-cotangent-dk)."""
    orders = np.asarray(orders, np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum([_psd_rows(int(p)) for p in orders])[:-1]])
    offsets = np.asarray(offsets, np.int64)
    gin = torch.empty_like(gout)
    ws = _proj_ws(len(orders), orders, gout.device)
    st = L.lib().psd_proj_vjp(len(orders), orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dt_code(gout.dtype),
                              _ptr(eigvals), _ptr(eigvecs), _ptr(gout.contiguous()), _ptr(gin), _ptr(ws),
                              _stream(gout.device))
    L.check(st, "psd_proj_vjp")
    return gin


def psd_proj_vjp_rule(eigvals, eigvecs, gout: torch.Tensor, orders, rule: str = "dk", eps: float = 0.0,
                      offsets=None):
    """A comparison backward rule of psd_proj from its decomposition: "dk"
    (eq:psd-cotangent-dk), "naive" (eq:psd-cotangent as autograd forms it) or
    "tikhonov" (the naive rule for the projection of S + eps I)."""
    orders = np.asarray(orders, np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum([_psd_rows(int(p)) for p in orders])[:-1]])
    offsets = np.asarray(offsets, np.int64)
    gin = torch.empty_like(gout)
    ws = _proj_ws(len(orders), orders, gout.device)
    st = L.lib().psd_proj_vjp_rule(len(orders), orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dt_code(gout.dtype),
                                   int(L.PSD_RULES[rule]), float(eps), _ptr(eigvals), _ptr(eigvecs),
                                   _ptr(gout.contiguous()), _ptr(gin), _ptr(ws), _stream(gout.device))
    L.check(st, "psd_proj_vjp_rule")
    return gin


def policy_init(seed: int = 0, head_scale: float = 0.0, dtype=torch.float32, device="cuda:0") -> torch.Tensor:
    """Initial parameters of the learned policy, in the flat layout of
    cosmo_policy_forward (App. E's initialisation): the first two layers of
    each network ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)); the last layer zero,
    so the untrained policy is COSMO with fixed penalties (or, head_scale > 0,
    ~ U(-head_scale, head_scale)); the initial logits those of Table 2's
    penalties (100 on zero rows, 0.1 on nonnegative, SOC and PSD rows) and
    relaxation 1.6."""
    rng = np.random.default_rng(seed)
    hid, parts = 32, []
    for n_in in (7, 5):
        parts += [rng.uniform(-1, 1, n_in * hid) / np.sqrt(n_in), rng.uniform(-1, 1, hid) / np.sqrt(n_in),
                  rng.uniform(-1, 1, hid * hid) / np.sqrt(hid), rng.uniform(-1, 1, hid) / np.sqrt(hid)]
        parts += [rng.uniform(-head_scale, head_scale, hid + 1) if head_scale > 0 else np.zeros(hid + 1)]
    lmin, lmax = np.log(1e-3), np.log(1e3)
    t = (np.log(np.array([100.0, 0.1, 0.1, 0.1])) - lmin) / (lmax - lmin)
    parts += [np.log(t / (1 - t)), [np.log(0.8 / 0.2)]]
    theta = np.concatenate([np.asarray(q, np.float64).ravel() for q in parts])
    assert theta.size == L.COSMO_POLICY_PARAMS
    return torch.from_numpy(theta).to(dtype=dtype, device=device)


class NewtonSchulzProj:
    """The Newton-Schulz comparison rule (eq:newton-schulz) over a set of
    svec blocks: forward() projects and keeps every iterate in a device tape,
    vjp() runs the reverse pass through the unrolled products."""

    def __init__(self, orders, iters: int, dtype=torch.float32, device="cuda:0", offsets=None):
        self.orders = np.asarray(orders, np.int32)
        if offsets is None:
            offsets = np.concatenate([[0], np.cumsum([_psd_rows(int(p)) for p in self.orders])[:-1]])
        self.offsets = np.asarray(offsets, np.int64)
        self.iters, self.dtype, self.device = int(iters), dtype, torch.device(device)
        nb = L.lib().psd_ns_tape_size(len(self.orders), self._o(), _dt_code(dtype), self.iters)
        if nb == 0:
            raise L.CosmoError(L.COSMO_EINVAL, "psd_ns_tape_size", "invalid blocks, dtype or step count")
        self.tape = torch.empty(int(nb), dtype=torch.uint8, device=self.device)
        self._ready = False

    def _o(self):
        return self.orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))

    def _off(self):
        return self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        assert x.dtype == self.dtype and x.device == self.device
        out = torch.empty_like(x)
        st = L.lib().psd_proj_ns(len(self.orders), self._o(), self._off(), _dt_code(x.dtype), self.iters,
                                 _ptr(x.contiguous()), _ptr(out), _ptr(self.tape), _stream(x.device))
        L.check(st, "psd_proj_ns")
        self._ready = True
        return out

    def vjp(self, gout: torch.Tensor, gin: Optional[torch.Tensor] = None) -> torch.Tensor:
        if not self._ready:
            raise RuntimeError("NewtonSchulzProj.vjp needs a forward() first")
        gin = torch.empty_like(gout) if gin is None else gin
        st = L.lib().psd_proj_ns_vjp(len(self.orders), self._o(), self._off(), _dt_code(gout.dtype), self.iters,
                                     _ptr(gout.contiguous()), _ptr(gin), _ptr(self.tape), _stream(gout.device))
        L.check(st, "psd_proj_ns_vjp")
        return gin


def socp_proj(x: torch.Tensor, dims: Sequence[int], offsets=None):
    dims = np.asarray(dims, np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum(dims)[:-1]])
    offsets = np.asarray(offsets, np.int64)
    out = torch.empty_like(x)
    ws = _proj_ws(len(dims), dims, x.device)
    st = L.lib().socp_proj(len(dims), dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dt_code(x.dtype),
                           _ptr(x.contiguous()), _ptr(out), _ptr(ws), _stream(x.device))
    L.check(st, "socp_proj")
    return out


def socp_proj_vjp(x: torch.Tensor, gout: torch.Tensor, dims, offsets=None):
    dims = np.asarray(dims, np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum(dims)[:-1]])
    offsets = np.asarray(offsets, np.int64)
    gin = torch.empty_like(gout)
    ws = _proj_ws(len(dims), dims, x.device)
    st = L.lib().socp_proj_vjp(len(dims), dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dt_code(x.dtype),
                               _ptr(x.contiguous()), _ptr(gout.contiguous()), _ptr(gin), _ptr(ws),
                               _stream(x.device))
    L.check(st, "socp_proj_vjp")
    return gin
