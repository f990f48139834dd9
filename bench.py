"""Benchmark: batched forward + backward unrolled COSMO on one MI355X.

Workloads (synthetic stand-ins with the shapes of the paper's App. F
classes; `--workload`, default c4, the largest configuration that runs on
one GPU):

  c1  one max-cut SDP on G(20, 0.3), float64, K = 100, forward only,
      CG tolerance 1e-10
  c2  64 max-cut SDPs, orders p ~ U{30..100}, edge probability U(0.1, 0.5),
      float32, K = 50 with per-step, per-row rho^k and per-instance alpha^k,
      forward + loss + backward
  c3  32 Lovasz theta SDPs on random circulant graphs, n ~ U{64..200},
      float32, K = 50, forward + loss + backward
  c4  256 Huber-regression SOCPs (2000 x 500 Gaussian design, Student-t
      noise, 200 second-order cones of dimension 3-10), K = 40, forward +
      loss + backward; the design is passed once as a dense block placed at
      +G and -G and stored as float32 (the data are float32 numbers), the
      iteration runs in float64 (the default line; --dtype f32 runs it in
      float32 throughout)
  c5  128 covariance-steering SDPs (nx in {4..12}, nu = nx/2, T ~ U{30..100}),
      float32, K = 30, forward + loss + backward

One timed step = one pass of the whole unroll over the whole batch with
inputs resident in HBM.  Prints one JSON line: instance-iterations per
second (B K / time per step), peak HBM of the batched pass against the plain
forward (B sequential single-instance forward-only calls, no tape), the
roofline of the dominant kernel measured with HIP events recorded by the
library on the stream the kernel runs on, the float64 oracle's own
throughput on the host cores over a bounded sample (cpu_baseline), and the
error of the timed run against the oracle's full K-step runs of sampled
instances (rel_err_vs_oracle).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd unrolled COSMO iters/s & peak HBM vs plain fwd, at 1e-5 rel err"
PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic work of one PSD block of order p: 9 p^3 for a textbook symmetric
# eigendecomposition (eigenvectors included) + 2 p^3 for U max(L, 0) U'.
EIG_FLOPS_PER_P3 = 11.0
# The library's PSD order classes: lanes per Jacobi pair, largest order (per
# dtype for the last class) and the orders they hold.
EIG_CLASSES = {0: (4, "32", "orders <= 32"), 1: (8, "64", "orders 33-64"), 2: (8, "128", "orders 65-128"),
               3: (8, None, "orders above 128")}


def eig_kernel_name(cls: int, threads: int, f32: bool) -> str:
    """Instantiation of the eigensolve kernel that ran order class cls."""
    g, pmax, what = EIG_CLASSES[cls]
    pmax = pmax or ("200" if f32 else "140")
    return f"k_psd_eig<{'float' if f32 else 'double'},{threads},{g},{pmax}> ({what})"
EIG_PROFILE = os.path.join(ROOT, "profiles", "k_psd_eig_maxcut64_pmc.md")
# the eigensolve kernels are built from k_psd.hip and the shared tile helpers
EIG_SOURCE = [os.path.join(ROOT, "paper_2606_13825_amd", "csrc", "k_psd.hip"),
              os.path.join(ROOT, "paper_2606_13825_amd", "csrc", "mma_tiles.h")]
PCG_PROFILE = os.path.join(ROOT, "profiles", "k_pcg_huber256_pmc.md")
PCG_C5_PROFILE = os.path.join(ROOT, "profiles", "k_pcg_coop_covsteer128_pmc.md")
NS_PROFILE = os.path.join(ROOT, "profiles", "k_ns_gemm_appc_pmc.md")
NS_SOURCE = [os.path.join(ROOT, "paper_2606_13825_amd", "csrc", "k_ns.hip"),
             os.path.join(ROOT, "paper_2606_13825_amd", "csrc", "mma_tiles.h")]
APPB_PROFILE = os.path.join(ROOT, "profiles", "k_pcg_coop_appb_pmc.md")
PCG_SOURCE = [os.path.join(ROOT, "paper_2606_13825_amd", "csrc", "k_pcg.hip"),
              os.path.join(ROOT, "paper_2606_13825_amd", "csrc", "wave_ops.h")]


def psd_order_class(orders):
    o = np.asarray(orders)
    return np.where(o <= 32, 0, np.where(o <= 64, 1, np.where(o <= 128, 2, 3)))


def traffic_from_profile(profile, source, **match):
    """HBM bytes per dispatch of a kernel, from a committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a copy kernel of
    known size); None when there is none, when its keys (order class, CG
    form) differ from `match`, or when the kernel source has changed since the
    counters were taken.  `source` is one file or a list of files, hashed
    together in that order."""
    try:
        kv = {}
        with open(profile) as f:
            for line in f:
                if ":" in line and line[:1].isalpha():
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        h = hashlib.sha256()
        for src in ([source] if isinstance(source, str) else source):
            with open(src, "rb") as f:
                h.update(f.read())
        sha = h.hexdigest()
        if kv.get("source_sha256") != sha or any(int(kv.get(k, -1)) != int(v) for k, v in match.items()):
            return None
        return float(kv["traffic_bytes_per_dispatch"])
    except (OSError, KeyError, ValueError):
        return None


def pcg_bytes_per_iteration(inst, esz, gsz=None):
    """Algorithmic HBM bytes of one PCG iteration (one operator application)
    on one instance: the values and column indices of A and A' (one pass
    each) and of P, plus the vectors the iteration streams (p, t = rho A p,
    M p, x, r, z).  A dense block (meta["dense"]) counts once, rows x cols
    values, however many placements it has; the CSR remainder counts as
    above."""
    nnz_a = inst.A.nnz
    dense_bytes = 0
    d = (getattr(inst, "meta", None) or {}).get("dense")
    if d:
        A = inst.A.tocsr()
        for (r0, _) in d["place"]:
            nnz_a -= A[int(r0):int(r0) + d["rows"], d["col0"]:d["col0"] + d["cols"]].nnz
        dense_bytes = d["rows"] * d["cols"] * (gsz or esz)
    nnz_p = inst.P.nnz if inst.P is not None else 0
    return dense_bytes + 2 * nnz_a * (esz + 4) + nnz_p * (esz + 4) + esz * (6 * inst.n + 2 * inst.m)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _workload(name):
    import synth
    f32 = lambda xs: [x.astype(np.float32) for x in xs]
    if name == "c1":
        return dict(name="maxcut_sdp_G20p0.3_fp64_K100_forward", insts=[synth.c1_instance()], K=100, dtype="f64",
                    backward=False, cg_tol=1e-10, hyper="default", cpu_sample=1, cpu_steps=100, err_sample=0)
    if name == "c2":
        return dict(name="maxcut_sdp_batch64_p30-100_fp32_K50", insts=f32(synth.c2_batch()), K=50, dtype="f32",
                    backward=True, hyper="perturbed", seed=2, cpu_sample=16, cpu_steps=50, err_sample=0)
    if name == "c3":
        # cond(M) ~ 2e5 here (trace row, rho_eq n): a relative residual of 1e-8 admits solve errors of ~2e-3
        # against the exact solve, so the CG runs to 1e-10 (in float32 it then stops at the precision floor)
        return dict(name="lovasz_circulant_batch32_n64-200_fp32_K50", insts=f32(synth.c3_batch()), K=50,
                    dtype="f32", backward=True, hyper="default", cpu_sample=16, cpu_steps=10, err_sample=2,
                    cg_tol=1e-10)
    if name == "c4":
        # float64 iterations on float32 data: the design block (the traffic)
        # is stored as float32, losslessly, the vectors and sums are float64
        return dict(name="huber_socp_batch256_2000x500_200soc_f64_blockf32_K40", insts=f32(synth.c4_batch()),
                    K=40, dtype="f64", dense_f32=True, backward=True, hyper="default", cpu_sample=16, cpu_steps=2,
                    err_sample=2, cg_tol=1e-10, cg_max_iter=1000)
    if name == "c5":
        return dict(name="covsteer_sdp_batch128_nx4-12_T30-100_fp32_K30", insts=f32(synth.c5_batch()), K=30,
                    dtype="f32", backward=True, hyper="default", cpu_sample=16, cpu_steps=30, err_sample=0,
                    cg_max_iter=2000)
    raise SystemExit(f"unknown workload {name}")


def _hyper(wl):
    """rho [K, m] and alpha [K] per instance: the R1 defaults with alpha = 1.6,
    or (c2, per-iteration learnable hyperparameters) a seeded log-uniform
    perturbation of them with alpha^k ~ U(1.4, 1.8)."""
    import synth
    npdt = np.float32 if wl["dtype"] == "f32" else np.float64
    rhos, alphas = [], []
    rng = np.random.default_rng(1000 + wl.get("seed", 0))
    for inst in wl["insts"]:
        if wl["hyper"] == "perturbed":
            r, a = synth.perturbed_hyper(inst, wl["K"], rng)
        else:
            r, a = synth.default_rho(inst, wl["K"]), np.full(wl["K"], 1.6)
        rhos.append(r.astype(np.float32).astype(npdt))
        alphas.append(a.astype(np.float32).astype(npdt))
    return rhos, alphas


def _oracle_job(args):
    inst, rho, alpha, backward = args
    import oracle
    t0 = time.perf_counter()
    tape, (x, s, y) = oracle.unroll_forward(inst, rho, alpha)
    grho = galpha = None
    if backward:
        g = oracle.residual_loss_grad(inst, x, s, y)
        grho, galpha, *_ = oracle.unroll_backward(inst, tape, *g)
    return time.perf_counter() - t0, x, s, y, grho, galpha


def _floor_job(args):
    """One realisation of the oracle's float32 rounding model on one instance
    (the floor float32 storage alone sets on it)."""
    inst, rho, alpha, backward, resid, r = args
    import oracle
    return oracle.rounding_floor_runs(inst, rho, alpha, backward=backward, solve_resid=resid, which=(r,))[0]


def float32_floor(wl, rhos, alphas, idx, ref_runs):
    """Largest relative errors (iterates, gradients) of the rounding model's
    three realisations against the oracle's exact runs, over instances idx
    (ref_runs[j] is the exact run of idx[j]).  Solves stop at the float32 CG
    residual (1e-7, or the workload's tolerance if larger) except on the
    max-cut family, whose reduced matrix is diagonal."""
    import multiprocessing as mp
    resid = 0.0 if wl["name"].startswith("maxcut") else max(wl.get("cg_tol", 1e-8), 1e-7)
    jobs = [(wl["insts"][i], rhos[i].astype(np.float64), alphas[i].astype(np.float64), wl["backward"], resid, r)
            for i in idx for r in range(3)]
    # this process has initialised the GPU: the workers are fresh interpreters
    with mp.get_context("spawn").Pool(min(len(jobs), 12)) as pool:
        runs = pool.map(_floor_job, jobs)
    e_it = e_g = 0.0
    for j, (x, s, y, grho, galpha) in enumerate(runs):
        ref = ref_runs[j // 3]
        for a, b in zip((x, s, y), ref[1:4]):
            e_it = max(e_it, np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12))
        if wl["backward"]:
            e_g = max(e_g, np.linalg.norm(grho - ref[4]) / max(np.linalg.norm(ref[4]), 1e-12),
                      np.linalg.norm(galpha - ref[5]) / max(np.linalg.norm(ref[5]), 1e-12))
    return e_it, e_g


def cpu_baseline(wl, rhos, alphas, n_sample, steps, workers):
    """The float64 oracle, as it stands, on the first n_sample instances and
    the first `steps` unrolled steps, instance-parallel over `workers`
    single-threaded processes."""
    import multiprocessing as mp
    jobs = [(wl["insts"][i], rhos[i][:steps].astype(np.float64), alphas[i][:steps].astype(np.float64),
             wl["backward"]) for i in range(n_sample)]
    # runs before this process touches the GPU, so forked workers are plain CPU processes
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_job, jobs)
    return time.perf_counter() - t0, res


def start_error_leg(wl, rhos, alphas, n_err):
    """The oracle's full K-step runs (forward and, if timed, backward) of the
    first n_err instances, one process each, started before this process
    touches the GPU and collected after the timed GPU run; they give the
    error of that run against the oracle when the throughput sample covers
    fewer than K steps.  Returns (pool, async result)."""
    import multiprocessing as mp
    jobs = [(wl["insts"][i], rhos[i].astype(np.float64), alphas[i].astype(np.float64), wl["backward"])
            for i in range(n_err)]
    pool = mp.get_context("fork").Pool(n_err)
    return pool, pool.map_async(_oracle_job, jobs)


def _copy_calibration():
    import torch
    n = 64 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "dispatches": 5}))


def psd_rules_study(samples=100, orders=(10, 20, 40, 80, 160, 320), delta=1e-5, ns_iters=20, reps=5):
    """Backward cost of the PSD-projection rules against the matrix order (the
    appendix's timing experiment): `samples` matrices per order from the App.
    C sampler at gap `delta`, one batched call per rule, HIP events on the
    launching stream.  DK, the eigendecomposition rule and Tikhonov reuse one
    decomposition (orders the eigensolver takes, <= 200 in float32);
    Newton-Schulz runs `ns_iters` steps forward, then its reverse pass is
    timed.  Prints one JSON line."""
    import torch
    from paper_2606_13825_amd import NewtonSchulzProj, psd_proj, psd_proj_vjp_rule
    from synth import svec_of_dense
    from synth.workloads import appc_matrix
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(7)
    rows, ns_roof = [], None

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    for n in orders:
        mats = [appc_matrix(n, delta, rng)[0] for _ in range(samples)]
        x = np.concatenate([svec_of_dense(m) for m in mats]).astype(np.float32)
        g = rng.standard_normal(x.shape).astype(np.float32)
        xt, gt = torch.from_numpy(x).to(dev), torch.from_numpy(g).to(dev)
        ords = [n] * samples
        row = {"order": n}
        if n <= 200:
            row["eigh_fwd_ms"] = timed(lambda: psd_proj(xt, ords, max_sweeps=60))
            _, lam, U = psd_proj(xt, ords, max_sweeps=60)
            for rule, eps in (("dk", 0.0), ("naive", 0.0), ("tikhonov", 1e-3), ("tikhonov", 1e-6)):
                key = rule if rule != "tikhonov" else f"tikhonov_{eps:.0e}"
                row[f"{key}_bwd_ms"] = timed(lambda: psd_proj_vjp_rule(lam, U, gt, ords, rule=rule, eps=eps))
        ns = NewtonSchulzProj(ords, ns_iters, torch.float32, dev)
        row["ns_fwd_ms"] = timed(lambda: ns.forward(xt))
        gin = torch.empty_like(gt)
        row["ns_bwd_ms"] = timed(lambda: ns.vjp(gt, gin))
        # reverse pass: 4 products per step plus 2 at the output, 2 p^3 flops each
        flops = samples * (4 * ns_iters + 2) * 2.0 * n ** 3
        row["ns_bwd_tflops"] = flops / (row["ns_bwd_ms"] * 1e-3) / 1e12
        rows.append(row)
        ns_roof = {"kernel": "k_ns_gemm<float> (Newton-Schulz reverse pass)", "order": n, "bound": "mfma",
                   "achieved": row["ns_bwd_tflops"], "peak": 157.3, "unit": "TFLOP/s",
                   "frac": row["ns_bwd_tflops"] / 157.3,
                   "traffic": traffic_from_profile(NS_PROFILE, NS_SOURCE, order=n),
                   "traffic_per": "one k_ns_gemm launch (100 blocks) at this order; achieved is the "
                                  "reverse pass's product flops over its event-timed duration"}
        print(f"[bench] psd rules order {n}: " + ", ".join(f"{k}={v:.3f}" for k, v in row.items() if k != "order"),
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "PSD-projection backward time per batch by rule (App. C matrices)",
                      "unit": "ms", "higher_is_better": False, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"appc_delta{delta:g}_x{samples}", "samples": samples,
                                 "ns_iters": ns_iters, "reps": reps},
                      "rows": rows, "roofline": ns_roof}))


# CG tolerance of the App. B runs: the float32 CG then stops at the
# precision floor of its float64 true residual (as for the parity tests).
APPB_CG_TOL = 1e-10


DENSE_SOLVE_MAX_ELEMENTS = 2**31 - 1


def _appb_dense_baseline(kind, P, A, rho_row, b, q, xstar, dev, reps=1):
    """One of the appendix's dense comparison methods for the App. B solve,
    with PyTorch's dense solver and autograd (a measured baseline, not the
    library's path): 'direct' forms the saddle-point matrix of
    eq:cosmo_linear_system, 'indirect_full' the reduced matrix M of
    eq:cosmo_linear_system_reduced; both solve the first step from z = 0 and
    backpropagate the least-squares loss 1/2 ||x~ - x*||^2 to rho.  Returns
    peak HBM of forward + backward (bytes over the state before) and the
    backward time (HIP events, the mean of `reps`), or the error when the
    device runs out of memory."""
    import torch
    f32 = torch.float32
    n, m = A.shape[1], A.shape[0]
    sigma = 1e-6
    dim = n + m if kind == "direct" else n
    if dim * dim > DENSE_SOLVE_MAX_ELEMENTS:
        # a 75000^2 saddle-point solve (5.6e9 elements) faulted the GPU inside
        # the vendor dense solver; solves past a 32-bit element count are not run
        return {"error": "not run", "detail": f"the dense matrix would hold {dim * dim:.3g} elements, more than "
                                                f"the {DENSE_SOLVE_MAX_ELEMENTS} this study hands the dense solver"}
    torch.cuda.synchronize(dev)
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)
    base = torch.cuda.memory_allocated(dev)
    try:
        Ac = A.tocoo()
        Ad = torch.sparse_coo_tensor(np.vstack([Ac.row, Ac.col]), Ac.data.astype(np.float32), (m, n),
                                     device=dev).to_dense()
        pd = torch.from_numpy(P.diagonal().astype(np.float32)).to(dev)
        qd = torch.from_numpy(q.astype(np.float32)).to(dev)
        bd = torch.from_numpy(b.astype(np.float32)).to(dev)
        xs = torch.from_numpy(xstar.astype(np.float32)).to(dev)
        rho = torch.from_numpy(rho_row.astype(np.float32)).to(dev).requires_grad_(True)
        ms = 0.0
        for _ in range(reps):
            if kind == "direct":
                K = torch.zeros((n + m, n + m), dtype=f32, device=dev)
                K[:n, :n] = torch.diag(pd + sigma)
                K[:n, n:] = Ad.T
                K[n:, :n] = Ad
                K = K - torch.diag(torch.cat([torch.zeros(n, dtype=f32, device=dev), 1.0 / rho]))
                rhs = torch.cat([-qd, bd])
                xt = torch.linalg.solve(K, rhs)[:n]
            else:
                M = torch.diag(pd + sigma) + Ad.T @ (rho[:, None] * Ad)
                xi = -qd + Ad.T @ (rho * bd)
                xt = torch.linalg.solve(M, xi)
            loss = 0.5 * torch.sum((xt - xs) ** 2)
            cur = torch.cuda.current_stream(dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(cur)
            (g,) = torch.autograd.grad(loss, rho)
            e1.record(cur)
            e1.synchronize()
            ms += e0.elapsed_time(e1) / reps
            ok = bool(torch.isfinite(g).all())
            del g, loss, xt
        peak = torch.cuda.max_memory_allocated(dev) - base
        return {"peak_hbm_bytes": int(peak), "bwd_ms": ms, "finite": ok}
    except torch.cuda.OutOfMemoryError as e:
        return {"error": "out of memory", "detail": str(e).split("\n")[0][:200]}
    finally:
        torch.cuda.synchronize(dev)
        torch.cuda.empty_cache()


def appb_study(ns=(1000, 2000, 5000, 10000, 20000, 50000), reps=3, seed=8, dense_baselines=False):
    """Memory and time of the matrix-free backward against the problem size
    (the linear-solve backward experiment of App. B): one instance per size
    from the App. B sampler (diagonal P ~ U(0, 10), m = n/2, A 1 % dense,
    rho ~ U(0, 1), b ~ N(0, 1), q = -P x*), one unrolled step (K = 1,
    alpha = 1, nonnegative cone on the rows) through the library's forward,
    residual loss and backward, float32, cooperative CG over the whole chip
    (tolerance APPB_CG_TOL).
    Peak HBM = the peak of torch's allocations (problem data, tape,
    workspaces, outputs) over forward + loss + backward plus the plan's own
    device buffer; the backward alone is timed with HIP events.  The dense
    reduced matrix (n^2) and saddle-point matrix ((n + m)^2) that the paper's
    comparison methods form are reported by size, and with dense_baselines
    both methods run (PyTorch dense solve and autograd, float32) on the same
    instance: peak HBM and backward time.  Prints one JSON line."""
    import torch
    from paper_2606_13825_amd import CosmoBatch
    from synth import Cone, ConicInstance
    from synth.workloads import appb_instance
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    rng = np.random.default_rng(seed)
    rows = []
    # one untimed pass on a small instance first: the runtime's one-time
    # device allocations (code objects, first plan) stay out of the figures
    for n in (200,) + tuple(ns):
        P, A, rho_row, b, xstar = appb_instance(n, rng)
        m = A.shape[0]
        inst = ConicInstance(P=P.tocsr(), q=-(P @ xstar), A=A.tocsr(), b=b, cones=[Cone("nonneg", m)])
        inst = inst.astype(np.float32)
        torch.cuda.synchronize(dev)
        torch.cuda.empty_cache()
        free0, res0 = torch.cuda.mem_get_info(dev)[0], torch.cuda.memory_reserved(dev)
        torch.cuda.reset_peak_memory_stats(dev)
        base = torch.cuda.memory_allocated(dev)
        batch = CosmoBatch([inst], K=1, dtype=torch.float32, device=dev, cg_tol=APPB_CG_TOL)
        torch.cuda.synchronize(dev)
        plan_bytes = max(0, (free0 - torch.cuda.mem_get_info(dev)[0]) - (torch.cuda.memory_reserved(dev) - res0))
        batch.set_pcg_form(4)
        rho = torch.from_numpy(rho_row.astype(np.float32)[None, :].copy()).to(dev)
        alpha = torch.ones((1, 1), dtype=torch.float32, device=dev)
        tape, fws, bws = batch.new_tape(), batch.new_fwd_ws(), batch.new_bwd_ws()
        stats = batch.new_stats()
        fw = batch.forward(rho, alpha, tape=tape, ws=fws, stats=stats)
        _, g = batch.residual_loss(fw.x, fw.s, fw.y, ws=fws)
        bw = batch.backward(rho, alpha, fw.tape, *g, ws=bws, stats=stats)
        torch.cuda.synchronize(dev)
        peak = torch.cuda.max_memory_allocated(dev) - base + plan_bytes
        assert torch.isfinite(bw.grho).all(), "non-finite gradient"
        st2 = batch.new_stats()
        out = (bw.grho, bw.galpha, bw.gx0, bw.gs0, bw.gy0)
        cur = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        for _ in range(reps):
            batch.backward(rho, alpha, fw.tape, *g, ws=bws, stats=st2, out=out)
        e1.record(cur)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        sd = batch.stats_dict(st2)
        ops = float(sd["cg_iters_total"].sum() + sd["cg_passes_total"].sum()) / reps
        cg_bytes = ops * pcg_bytes_per_iteration(inst, 4)
        row = {"n": n, "m": m, "nnz_A": int(inst.A.nnz), "peak_hbm_bytes": int(peak), "plan_bytes": int(plan_bytes),
               "bwd_ms": ms, "bwd_cg_operator_applications": ops, "bwd_cg_bytes": cg_bytes,
               "bwd_cg_gbs": cg_bytes / (ms * 1e-3) / 1e9,
               "dense_reduced_matrix_bytes": 4 * n * n, "dense_kkt_bytes": 4 * (n + m) ** 2}
        # every plan is destroyed here, on a synchronised device, not at interpreter exit
        torch.cuda.synchronize(dev)
        batch.close()
        del batch, tape, fws, bws, fw, bw, g, out
        if n == 200:
            continue
        if dense_baselines:
            for kind in ("indirect_full", "direct"):
                row[kind] = _appb_dense_baseline(kind, P, A.tocsr(), rho_row, b, -(P @ xstar), xstar, dev)
                print(f"[bench] appb n={n} {kind}: {row[kind]}", file=sys.stderr, flush=True)
        rows.append(row)
        print(f"[bench] appb n={n}: peak {peak / 2**20:.1f} MiB, backward {ms:.2f} ms, "
              f"{ops:.0f} operator applications, {row['bwd_cg_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    torch.cuda.synchronize(dev)
    last = rows[-1]
    print(json.dumps({"metric": "peak HBM and backward time of the matrix-free backward vs problem size (App. B)",
                      "unit": "bytes, ms", "higher_is_better": False, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "appb_one_instance_per_size", "sizes": list(ns), "K": 1,
                                 "pcg_form": 4, "cg_tol": APPB_CG_TOL, "reps": reps,
                                 "dense_baselines": dense_baselines},
                      "rows": rows,
                      "roofline": {"kernel": "k_pcg_coop<float> (backward adjoint solve)", "n": last["n"],
                                   "bound": "hbm", "achieved": last["bwd_cg_gbs"], "peak": PEAK_HBM_GBS,
                                   "unit": "GB/s", "frac": last["bwd_cg_gbs"] / PEAK_HBM_GBS,
                                   "traffic": traffic_from_profile(APPB_PROFILE, PCG_SOURCE, n=last["n"]),
                                   "traffic_per": "one backward adjoint solve (one k_pcg_coop launch)"}}))


def psd_trajectory_study(K=100, seed=5, alpha=1.6, ns_iters=40, fd_rel_step=1e-6):
    """The PSD-backward rules along a real COSMO trajectory (Fig. 3 and its
    appendix): the double-integrator covariance-steering SDP (N = 10, one PSD
    block of order 44), K steps in float64 at the default penalties and fixed
    alpha, from a standard-normal (x0, s0, y0), the final-residual loss, and
    one backward pass with the per-step tap on: at each step k the matrix S_k
    the solver projects (v^k on the PSD rows) and the cotangent Tbar_k the
    reverse pass delivers to the projection's output.  Every rule is applied
    to that pair, in float64 and in float32 (S_k and Tbar_k rounded): DK
    (eq:psd-cotangent-dk), the eigendecomposition rule as autograd forms it
    (eq:psd-cotangent), Tikhonov at eps 1e-3 and 1e-6, and Newton-Schulz
    (eq:newton-schulz, ns_iters steps, reverse pass through them).  Per step:
    Frobenius norm of each rule's Sbar_k (the svec 2-norm), whether it is
    finite, its relative distance from the float64 DK result, the minimum
    eigenvalue gap of S_k, and the true directional derivative
    <Tbar_k, dPi(S_k)[E]> by a central difference of the float64 projection
    along a random unit E (step fd_rel_step max(1, ||S_k||)) against each
    rule's <Sbar_k, E>.  Prints one JSON line."""
    import torch
    from paper_2606_13825_amd import CosmoBatch, NewtonSchulzProj, psd_proj, psd_proj_vjp_rule
    from synth import cone_row_slices, default_rho, double_integrator_cs
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    inst = double_integrator_cs(rng)
    (psd_cone, rows), = [(c, sl) for c, sl in cone_row_slices(inst.cones) if c.kind == "psd"]
    p = psd_cone.size
    batch = CosmoBatch([inst], K=K, dtype=torch.float64, device=dev, cg_tol=1e-12, cg_max_iter=2000)
    rho = torch.from_numpy(default_rho(inst, K)).to(dev)
    al = torch.full((K, 1), alpha, dtype=torch.float64, device=dev)
    z0 = [torch.from_numpy(rng.standard_normal(d)).to(dev) for d in (inst.n, inst.m, inst.m)]
    stats = batch.new_stats()
    fw = batch.forward(rho, al, *z0, stats=stats)
    loss, g = batch.residual_loss(fw.x, fw.s, fw.y)
    tap = torch.zeros((K, 2, inst.m), dtype=torch.float64, device=dev)
    batch.set_tap(tap)
    bw = batch.backward(rho, al, fw.tape, *g, stats=stats)
    batch.set_tap(None)
    torch.cuda.synchronize(dev)
    sd = batch.stats_dict(stats)
    S = tap[:, 0, rows].contiguous().view(-1)
    T = tap[:, 1, rows].contiguous().view(-1)
    orders = [p] * K
    nr = p * (p + 1) // 2

    def per_block_norm(v):
        return torch.linalg.vector_norm(v.view(K, nr).double(), dim=1).cpu().numpy()

    def apply_rules(Sd, Td, dt):
        Sx, Tx = Sd.to(dt).contiguous(), Td.to(dt).contiguous()
        _, lam, U = psd_proj(Sx, orders, max_sweeps=60)
        out = {}
        for key, rule, eps in (("dk", "dk", 0.0), ("autograd", "naive", 0.0),
                               ("tikhonov_1e-03", "tikhonov", 1e-3), ("tikhonov_1e-06", "tikhonov", 1e-6)):
            out[key] = psd_proj_vjp_rule(lam, U, Tx, orders, rule=rule, eps=eps)
        ns = NewtonSchulzProj(orders, ns_iters, dt, dev)
        pns = ns.forward(Sx)
        out["newton_schulz"] = ns.vjp(Tx)
        return out, lam, pns

    proj64, lam64, _ = psd_proj(S, orders, max_sweeps=60)
    r64, _, pns64 = apply_rules(S, T, torch.float64)
    r32, _, _ = apply_rules(S, T, torch.float32)
    # the true directional derivative of <Tbar, Pi(.)> at S_k along a random unit E
    E = torch.from_numpy(rng.standard_normal((K, nr))).to(dev)
    E = (E / torch.linalg.vector_norm(E, dim=1, keepdim=True)).view(-1)
    h = fd_rel_step * np.maximum(1.0, per_block_norm(S))
    hv = torch.from_numpy(np.repeat(h, nr)).to(dev)
    pp, _, _ = psd_proj(S + hv * E, orders, max_sweeps=60, want_eig=False)
    pm, _, _ = psd_proj(S - hv * E, orders, max_sweeps=60, want_eig=False)
    fd = ((T * (pp - pm)).view(K, nr).sum(1) / torch.from_numpy(2 * h).to(dev)).cpu().numpy()
    lam_np = lam64.view(K, p).cpu().numpy()
    lam_sorted = np.sort(lam_np, axis=1)
    gaps = np.diff(lam_sorted, axis=1).min(axis=1)
    dk64 = r64["dk"].view(K, nr)
    dk_norm = per_block_norm(r64["dk"])
    steps = []
    for k in range(K):
        row = {"k": k, "min_eig_gap": float(gaps[k]), "min_abs_eig": float(np.abs(lam_np[k]).min()),
               "n_negative": int((lam_np[k] < 0).sum()), "cotangent_norm": float(per_block_norm(T)[k]),
               "S_norm": float(per_block_norm(S)[k]), "fd_directional": float(fd[k]),
               "ns_forward_rel_err": float(torch.linalg.vector_norm((pns64 - proj64).view(K, nr)[k]) /
                                           max(float(torch.linalg.vector_norm(proj64.view(K, nr)[k])), 1e-300))}
        for prec, res in (("f64", r64), ("f32", r32)):
            for key, gin in res.items():
                gk = gin.view(K, nr)[k].double()
                fin = bool(torch.isfinite(gk).all())
                nrm = float(torch.linalg.vector_norm(gk)) if fin else None
                dirv = float((gk * E.view(K, nr)[k]).sum()) if fin else None
                row[f"{key}_{prec}"] = {
                    "norm": nrm, "finite": fin,
                    "rel_to_dk_f64": (float(torch.linalg.vector_norm(gk - dk64[k])) / max(dk_norm[k], 1e-300))
                    if fin else None,
                    "fd_rel_err": abs(dirv - fd[k]) / max(abs(fd[k]), 1e-12 * row["cotangent_norm"], 1e-300)
                    if fin else None}
        steps.append(row)
    summary = {}
    for prec in ("f64", "f32"):
        for key in r64:
            nm = f"{key}_{prec}"
            bad = [s["k"] for s in steps if not s[nm]["finite"]]
            fin = [s for s in steps if s[nm]["finite"]]
            summary[nm] = {"nonfinite_steps": len(bad), "first_nonfinite_step": bad[0] if bad else None,
                           "max_rel_to_dk_f64": max((s[nm]["rel_to_dk_f64"] for s in fin), default=None),
                           "median_fd_rel_err": float(np.median([s[nm]["fd_rel_err"] for s in fin])) if fin else None}
        print(f"[bench] psd trajectory {prec}: " + "; ".join(
            f"{key} nonfinite {summary[f'{key}_{prec}']['nonfinite_steps']}/{K}" for key in r64),
            file=sys.stderr, flush=True)
    batch.close()
    print(json.dumps({"metric": "PSD-projection backward rules along a COSMO trajectory (Fig. 3)",
                      "unit": "Frobenius norm per step", "higher_is_better": None, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"double_integrator_cs_N10_psd{p}_K{K}", "n": inst.n, "m": inst.m,
                                 "psd_order": p, "K": K, "alpha": alpha, "ns_iters": ns_iters, "seed": seed,
                                 "rho": "default penalties (zero-cone rows 100, others 0.1)",
                                 "z0": "standard normal", "loss": "final residual"},
                      "loss": float(loss[0]), "grad_alpha_norm": float(torch.linalg.vector_norm(bw.galpha)),
                      "cg_iters_max": int(sd["cg_iters_max"][0]), "nonfinite": int(sd["nonfinite"][0]),
                      "eig_not_converged": int(sd["eig_not_converged"][0]),
                      "min_eig_gap_first_last": [float(gaps[0]), float(gaps[-1])],
                      "summary": summary, "steps": steps}))


# Algorithmic flops per row of one reverse pass of the penalty network
# (k_pol_rho_bwd): the forward recomputed (X W1' over 8 inputs, H1 W2, the
# head) and the reverse (head, W2-bar = H1' H2-bar, H1-bar = H2-bar W2',
# W1'-bar = X' H1-bar, the 7 feature cotangents), 2 flops per multiply-add.
POLICY_BWD_FLOPS_PER_ROW = 2 * (8 * 32 + 32 * 32 + 32) + 2 * (32 + 32 * 32 + 32 * 32 + 8 * 32 + 7 * 32)


def policy_study(workload="c2", reps=3, head_scale=0.05, seed=3):
    """Cost of the learned policy inside the unroll (App. E): on the batch of
    `workload`, one forward + backward pass with the policy choosing rho^k and
    alpha^k at every step (cosmo_policy_forward / cosmo_policy_backward, the
    log-residual loss) against the same batch with fixed penalties
    (cosmo_unroll_forward, final-residual loss, cosmo_unroll_backward), HIP
    events on the stream, mean of `reps` after one untimed pass.  No trained
    weights exist: the parameters are App. E's initialisation with the last
    layers drawn from U(-head_scale, head_scale) so the penalties move.
    Prints one JSON line."""
    import torch
    from paper_2606_13825_amd import CosmoBatch, policy_init
    wl = _workload(workload)
    dev = torch.device("cuda:0")
    tdt = torch.float32 if wl["dtype"] == "f32" else torch.float64
    batch = CosmoBatch(wl["insts"], K=wl["K"], dtype=tdt, device=dev, cg_tol=wl.get("cg_tol"),
                       cg_max_iter=wl.get("cg_max_iter", 500), dense_f32=wl.get("dense_f32", False))
    theta = policy_init(seed, head_scale, tdt, dev)
    rhos, alphas = _hyper(wl)
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(dev)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(dev)
    tape, fws, bws = batch.new_tape(), batch.new_fwd_ws(), batch.new_bwd_ws()
    pt, pw = batch.policy_sizes()
    ptape = torch.empty(pt, dtype=torch.uint8, device=dev)
    pws = torch.empty(pw, dtype=torch.uint8, device=dev)
    stats = batch.new_stats()

    def fixed():
        fw = batch.forward(rho, alpha, tape=tape, ws=fws, stats=stats)
        _, g = batch.residual_loss(fw.x, fw.s, fw.y, ws=fws)
        batch.backward(rho, alpha, fw.tape, *g, ws=bws, stats=stats)

    out = {}

    def policy():
        fw = batch.policy_forward(theta, tape=tape, ptape=ptape, pws=pws, ws=fws, stats=stats)
        out["fw"] = fw
        out["g"] = batch.policy_backward(theta, fw, ws=bws, stats=stats)

    def timed(fn):
        fn()
        torch.cuda.synchronize(dev)
        cur = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        for _ in range(reps):
            fn()
        e1.record(cur)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_fixed = timed(fixed)
    ms_policy = timed(policy)
    fw, g = out["fw"], out["g"]
    rho_k = fw.rho.double()
    sd = batch.stats_dict(stats)
    row = {"fixed_fwd_bwd_ms": ms_fixed, "policy_fwd_bwd_ms": ms_policy,
           "policy_overhead": ms_policy / ms_fixed - 1.0,
           "policy_loss_mean": float(fw.loss.double().mean()),
           "rho_range": [float(rho_k.min()), float(rho_k.max())],
           "alpha_range": [float(fw.alpha.min()), float(fw.alpha.max())],
           "gtheta_norm": float(torch.linalg.vector_norm(g[0].double())),
           "gtheta_finite": bool(torch.isfinite(g[0]).all()), "nonfinite": int(sd["nonfinite"].max())}
    print(f"[bench] policy study {workload}: " + ", ".join(f"{k}={v}" for k, v in row.items()), file=sys.stderr,
          flush=True)
    print(json.dumps({"metric": "fwd+bwd unrolled COSMO with the learned policy vs fixed penalties (App. E)",
                      "unit": "ms per pass", "higher_is_better": False, "dtype": wl["dtype"], "data": "synthetic",
                      "config": {"workload": wl["name"], "K": wl["K"], "B": len(wl["insts"]), "reps": reps,
                                 "m_tot": batch.m_tot, "n_tot": batch.n_tot, "head_scale": head_scale,
                                 "policy_bwd_flops_per_row": POLICY_BWD_FLOPS_PER_ROW},
                      "result": row}))
    batch.close()


def vanilla_study(workload="c2", max_iter=4000, check=1):
    """The vanilla baseline of Sec. "Experiments": every instance of
    `workload` solved to eps = 1e-3 (absolute and relative) by COSMO with the
    residual-balancing penalty (cosmo_solve; zero start, alpha = 1.6, one
    penalty scalar per instance starting at 0.1, x 1e3 on zero rows), the
    whole batch in one call, checked every `check` steps.  Reports the steps
    to tolerance per instance (median, quartiles), the batch's wall-clock
    time (HIP events) and time per step.  Prints one JSON line."""
    import torch
    from paper_2606_13825_amd import CosmoBatch
    wl = _workload(workload)
    dev = torch.device("cuda:0")
    tdt = torch.float32 if wl["dtype"] == "f32" else torch.float64
    batch = CosmoBatch(wl["insts"], K=check, dtype=tdt, device=dev, cg_tol=wl.get("cg_tol"),
                       cg_max_iter=wl.get("cg_max_iter", 500), dense_f32=wl.get("dense_f32", False))
    stats = batch.new_stats()
    cur = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    e0.record(cur)
    iters, rho, x, s, y = batch.solve(max_iter=max_iter, stats=stats)
    e1.record(cur)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    ok = iters[iters > 0]
    steps = int(iters.max()) if np.all(iters > 0) else max_iter
    row = {"instances": int(len(iters)), "converged": int((iters > 0).sum()),
           "iters_median": float(np.median(ok)) if ok.size else None,
           "iters_q1_q3": [float(np.percentile(ok, 25)), float(np.percentile(ok, 75))] if ok.size else None,
           "iters_max": int(ok.max()) if ok.size else None, "batch_steps": steps, "batch_ms": ms,
           "ms_per_step": ms / steps, "rho_final_median": float(np.median(rho)),
           "cg_not_converged": int(batch.stats_dict(stats)["cg_not_converged"].sum())}
    print(f"[bench] vanilla {workload}: " + ", ".join(f"{k}={v}" for k, v in row.items()), file=sys.stderr,
          flush=True)
    print(json.dumps({"metric": "steps and time to eps = 1e-3, COSMO with residual balancing (vanilla baseline)",
                      "unit": "steps, ms", "higher_is_better": False, "dtype": wl["dtype"], "data": "synthetic",
                      "config": {"workload": wl["name"], "B": len(wl["insts"]), "check_every": check,
                                 "max_iter": max_iter, "eps_abs": 1e-3, "eps_rel": 1e-3, "rho0": 0.1,
                                 "eq_scale": 1e3, "alpha": 1.6, "interval": 40, "tol_factor": 5},
                      "result": row, "iters": iters.tolist()}))
    batch.close()


def scp_study(scenarios=20, horizon=10, seed=11, eps=1e-6, check=10, max_outer=30, inner_max=20000, cg_tol=1e-12):
    """Sequential convex programming for the unicycle of App. F (Fig. 1's
    setting: 20 sampled scenarios, SCP tolerance 1e-3 on the nonlinear
    defect and the virtual control; horizon 10 by default, the
    standalone-results table's 20 or the appendix's 30 with --scp-horizon,
    at several times the cost per step), every
    convex step solved by the vanilla COSMO on the GPU to `eps` (float64,
    stopping test every `check` steps), all scenarios advancing together in
    one super-batch per outer iteration.  The CG runs to `cg_tol` relative:
    with the table caption's 1e-8 the inexact solves leave ADMM short of
    eps = 1e-6 on some of these programs, which then run to `inner_max`.  Reports per scenario the outer iterations and inner
    steps, the median and quartiles of the SCP residual max(|defect|, |nu|)
    against the outer iteration, and where the wall-clock time went (host
    assembly, upload, GPU solve, host ratio tests).  Prints one JSON line."""
    import torch
    from paper_2606_13825_amd.scp import scp_solve, ScpTiming
    from synth.covsteer import (unicycle_scenario, unicycle_subproblem, unicycle_initial_reference, unicycle_step,
                                unicycle_jacobians, unpack_solution, UNICYCLE_DT)
    rng = np.random.default_rng(seed)
    scs = [unicycle_scenario(rng, N=horizon) for _ in range(scenarios)]
    tm = ScpTiming()
    dev = torch.device("cuda:0")
    print(f"[bench] scp: {scenarios} unicycle scenarios, N={horizon}, inner eps={eps}, check every {check}",
          file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    res = scp_solve(scs, step=lambda x, u: unicycle_step(x, u, UNICYCLE_DT),
                    jacobians=lambda x, u: unicycle_jacobians(x, u, UNICYCLE_DT), subproblem=unicycle_subproblem,
                    unpack=unpack_solution, reference=unicycle_initial_reference, eps=eps, check=check,
                    max_outer=max_outer, inner_max=inner_max, dtype=torch.float64, device=dev, timing=tm,
                    cg_tol=cg_tol,
                    progress=lambda r, n, dt, it: print(f"[bench] scp outer {r}: {n} scenarios, {dt:.2f}s, "
                                                        f"inner steps median {int(np.median(it))} max {int(it.max())}"
                                                        f", {int((it < 0).sum())} at the step budget",
                                                        file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    ok = [r for r in res if r.converged]
    outers = np.array([r.outer for r in ok]) if ok else np.zeros(0)
    # the SCP residual max(|defect|, |nu|) of the current reference after each
    # outer iteration (nan before the first accepted step; a finished
    # scenario keeps its last value)
    C = np.full((len(res), max(r.outer for r in res)), np.nan)
    for i, r in enumerate(res):
        cur = np.nan
        for j, h in enumerate(r.history):
            if h.accepted:
                cur = max(h.defect, h.nu)
            C[i, j] = cur
        C[i, r.outer:] = cur
    conv = {"median": np.nanmedian(C, axis=0).tolist(), "q1": np.nanpercentile(C, 25, axis=0).tolist(),
            "q3": np.nanpercentile(C, 75, axis=0).tolist()}
    row = {"scenarios": scenarios, "converged": len(ok),
           "outer_median": float(np.median(outers)) if ok else None,
           "outer_q1_q3": [float(np.percentile(outers, 25)), float(np.percentile(outers, 75))] if ok else None,
           "inner_total_median": float(np.median([r.inner_total for r in res])),
           "wall_s": wall, "wall_s_per_scenario": wall / scenarios, "gpu_solve_s": tm.solve_s,
           "host_build_s": tm.build_s, "upload_s": tm.upload_s, "host_ratio_s": tm.host_s, "rounds": tm.rounds}
    print(f"[bench] scp: " + ", ".join(f"{k}={v}" for k, v in row.items()), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "SCP outer iterations and time to the 1e-3 SCP residual, unicycle covariance "
                                "steering, convex steps by vanilla COSMO on the GPU",
                      "unit": "iterations, s", "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"unicycle covariance steering, {scenarios} scenarios, N={horizon}",
                                 "inner_eps": eps, "cg_tol": cg_tol, "check_every": check, "max_outer": max_outer,
                                 "inner_max": inner_max, "seed": seed},
                      "result": row, "residual_curve": conv,
                      "per_scenario": [{"converged": r.converged, "outer": r.outer, "inner_total": r.inner_total,
                                        "inner": [h.inner for h in r.history],
                                        "accepted": [h.accepted for h in r.history]} for r in res]}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--cpu-sample", type=int, default=None, help="instances in the oracle sample")
    ap.add_argument("--dtype", default=None, choices=["f32"],
                    help="f32: run the workload in float32 throughout (dense blocks, vectors, sums)")
    ap.add_argument("--plain-sample", type=int, default=32,
                    help="instances timed in the plain (unbatched forward-only) comparison")
    ap.add_argument("--schedule", default="auto", choices=["auto", "eager0"],
                    help="auto: the autotuner's choice; eager0: CG form 0, eager launches")
    ap.add_argument("--psd-threads", default=None,
                    help="with --schedule eager0: eigensolve threads per order class and DK VJP threads, "
                         "five comma-separated numbers (e.g. 128,512,1024,1024,1024); default: the class defaults")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-floor", action="store_true",
                    help="skip the float32 floor of the error sample (the oracle's rounding model)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (unbatched forward-only) comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB five times (reference for the HBM byte counters)")
    ap.add_argument("--quick", action="store_true",
                    help="counter-collection run: the timed steps only (no plain-forward comparison, "
                         "no event-timed step, no CPU leg)")
    ap.add_argument("--dense-baselines", action="store_true",
                    help="with --study appb: also run the dense Direct and Indirect-Full backward passes")
    ap.add_argument("--study", default=None,
                    choices=["psd_rules", "appb", "psd_trajectory", "policy", "vanilla", "scp"],
                    help="psd_rules: backward time of the PSD-projection rules against the matrix order; "
                         "appb: peak HBM and time of the matrix-free backward against the problem size; "
                         "psd_trajectory: the PSD-projection backward rules along a COSMO trajectory; "
                         "policy: the learned policy's cost inside the unroll (on --workload); "
                         "vanilla: steps and time to eps = 1e-3 with residual balancing (on --workload); "
                         "scp: sequential convex programming for the unicycle, convex steps by vanilla COSMO")
    ap.add_argument("--scp-horizon", type=int, default=10, help="with --study scp: the horizon N")
    ap.add_argument("--scp-scenarios", type=int, default=20, help="with --study scp: the number of scenarios")
    ap.add_argument("--scp-cg-tol", type=float, default=1e-12, help="with --study scp: the CG relative tolerance")
    ap.add_argument("--scp-max-outer", type=int, default=30, help="with --study scp: outer iterations at most")
    args = ap.parse_args()
    if args.study == "psd_rules" and args.gpus == 1:
        psd_rules_study()
        return
    if args.study == "appb" and args.gpus == 1:
        appb_study(dense_baselines=args.dense_baselines)
        return
    if args.study == "psd_trajectory" and args.gpus == 1:
        psd_trajectory_study()
        return
    if args.study == "policy" and args.gpus == 1:
        policy_study(args.workload)
        return
    if args.study == "scp" and args.gpus == 1:
        scp_study(scenarios=args.scp_scenarios, horizon=args.scp_horizon, cg_tol=args.scp_cg_tol,
                  max_outer=args.scp_max_outer)
        return
    if args.study == "vanilla" and args.gpus == 1:
        vanilla_study(args.workload)
        return
    if args.quick:
        args.no_cpu_baseline = True
        args.no_plain = True
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU: the batch shards over instances with no "
                                   "exchange inside the unroll, but runs on more than one GPU are not part of it"}))
        raise SystemExit(2)
    if args.copy_calibration:
        _copy_calibration()
        return

    wl = _workload(args.workload)
    if args.dtype == "f32" and wl["dtype"] != "f32":
        wl = dict(wl, dtype="f32", name=wl["name"].replace("_f64_blockf32", "_fp32"))
        for key in ("dense_f32", "cg_tol"):
            wl.pop(key, None)
    insts, K, backward = wl["insts"], wl["K"], wl["backward"]
    B = len(insts)
    rhos, alphas = _hyper(wl)
    print(f"[bench] workload {wl['name']}: B={B} K={K}", file=sys.stderr, flush=True)

    cpu = None
    err_leg = None
    if not args.no_cpu_baseline:
        try:
            aff = len(os.sched_getaffinity(0))
        except AttributeError:
            aff = os.cpu_count() or 1
        aff = min(16, aff)
        n_s = min(args.cpu_sample or wl["cpu_sample"], B)
        steps = min(wl["cpu_steps"], K)
        n_err = min(wl["err_sample"], B) if steps < K else 0
        if n_err:
            err_leg = (start_error_leg(wl, rhos, alphas, n_err), n_err)
            print(f"[bench] error leg: oracle runs of {n_err} instances x {K} steps started", file=sys.stderr,
                  flush=True)
        workers = max(1, min(aff - n_err, n_s))
        wall, res = cpu_baseline(wl, rhos, alphas, n_s, steps, workers)
        cpu = (wall, res, workers, n_s, steps)
        print(f"[bench] cpu baseline: {n_s} instances x {steps} steps in {wall:.1f} s on {workers} processes",
              file=sys.stderr, flush=True)

    import torch
    from paper_2606_13825_amd import CosmoBatch

    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)          # initialise the device before the memory counters
    tdt = torch.float32 if wl["dtype"] == "f32" else torch.float64
    kw = {}
    for key in ("cg_tol", "cg_max_iter", "dense_f32"):
        if key in wl:
            kw[key] = wl[key]

    torch.cuda.synchronize(dev)
    torch.cuda.reset_peak_memory_stats(dev)
    base_mem = torch.cuda.memory_allocated(dev)
    free0, res0 = torch.cuda.mem_get_info(dev)[0], torch.cuda.memory_reserved(dev)
    batch = CosmoBatch(insts, K=K, dtype=tdt, device=dev, **kw)
    torch.cuda.synchronize(dev)
    # the plan's own device buffer (transposed CSR, descriptors, maps): the
    # device's free memory fell by more than torch reserved
    plan_bytes = max(0, (free0 - torch.cuda.mem_get_info(dev)[0]) - (torch.cuda.memory_reserved(dev) - res0))
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(dev)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(dev)
    tape = batch.new_tape() if backward else None
    fws = batch.new_fwd_ws()
    bws = batch.new_bwd_ws() if backward else None
    stats = batch.new_stats()
    # fixed output buffers: every step passes the same pointers (a graph-mode
    # plan then replays its recording instead of recording again)
    vec = lambda n: torch.empty(n, dtype=tdt, device=dev)
    fout = (vec(batch.n_tot), vec(batch.m_tot), vec(batch.m_tot))
    seeds = (vec(batch.n_tot), vec(batch.m_tot), vec(batch.m_tot))
    bout = (torch.empty((K, batch.m_tot), dtype=tdt, device=dev), torch.empty((K, batch.B), dtype=tdt, device=dev),
            vec(batch.n_tot), vec(batch.m_tot), vec(batch.m_tot))

    def step():
        if not backward:
            return batch.forward(rho, alpha, tape=False, ws=fws, stats=stats, out=fout), None, None
        fw = batch.forward(rho, alpha, tape=tape, ws=fws, stats=stats, out=fout)
        loss, g = batch.residual_loss(fw.x, fw.s, fw.y, ws=fws)
        for dst, src in zip(seeds, g):
            dst.copy_(src)
        bw = batch.backward(rho, alpha, fw.tape, *seeds, ws=bws, stats=stats, out=bout)
        return fw, loss, bw

    # the project's autotuner fixes the schedule (CG form, graph replay or
    # eager launches) before anything is timed; --schedule eager0 pins CG form
    # 0 with eager launches (the form the counter summaries were taken with)
    if args.schedule == "auto":
        form, ms = batch.autotune(rho, alpha, fws)
        sched = {"pcg_form": form, "graph": batch.graph(),
                 "autotune_forward_ms": dict(zip(("form0", "form2", "form4", "form0_graph"), ms))}
        if any(c.kind == "psd" for inst in insts for c in inst.cones):
            eig, vjp = batch.psd_schedule()
            sched.update({"eig_threads_per_class": eig, "vjp_threads": vjp, "autotune_psd_ms": batch.psd_tune_ms()})
    else:
        batch.set_graph(False)
        batch.set_pcg_form(0)
        sched = {"pcg_form": 0, "graph": False, "autotune_forward_ms": None}
        if args.psd_threads:
            t = [int(v) for v in args.psd_threads.split(",")]
            if len(t) != 5:
                raise SystemExit("--psd-threads takes five numbers: four order classes and the VJP")
            batch.set_psd_schedule(t[:4], t[4])
        if any(c.kind == "psd" for inst in insts for c in inst.cones):
            eig, vjp = batch.psd_schedule()
            sched.update({"eig_threads_per_class": eig, "vjp_threads": vjp})
    print(f"[bench] autotune: {sched}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fw, loss, bw = step()
    torch.cuda.synchronize(dev)
    dt = (time.perf_counter() - t0) / args.steps
    peak_fb = torch.cuda.max_memory_allocated(dev) - base_mem + plan_bytes
    print(f"[bench] {'fwd+bwd' if backward else 'fwd'} {dt * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    if args.quick:
        print(json.dumps({"metric": METRIC + " (counter-collection run)", "value": B * K / dt,
                          "unit": "instance-iterations/s", "ms_per_step": dt * 1e3,
                          "config": {"workload": wl["name"]}}))
        return

    # kernel families, and the eigensolve kernel of each PSD order class alone,
    # timed with HIP events recorded by the library on the streams they run on
    st_prof = batch.new_stats()
    batch.set_profiling(True)
    if backward:
        fw2 = batch.forward(rho, alpha, tape=tape, ws=fws, stats=st_prof)
        _, g2 = batch.residual_loss(fw2.x, fw2.s, fw2.y, ws=fws)
        batch.backward(rho, alpha, fw2.tape, *g2, ws=bws, stats=st_prof)
    else:
        batch.forward(rho, alpha, tape=False, ws=fws, stats=st_prof)
    torch.cuda.synchronize(dev)
    fam = {}
    for kind, name in ((0, "psd_eig_project"), (1, "psd_dk_vjp"), (2, "pcg"), (3, "csr_row_col_passes")):
        fam[name] = batch.profile_read(kind)
    cls = {c: batch.profile_read(4 + c) for c in range(4)}
    batch.set_profiling(False)
    sprof = batch.stats_dict(st_prof)
    print(f"[bench] kernel families (launches, ms): {fam}", file=sys.stderr, flush=True)
    print(f"[bench] eigensolve per order class (launches, ms): {cls}", file=sys.stderr, flush=True)

    rooflines = {}
    orders = np.array([c.size for inst in insts for c in inst.cones if c.kind == "psd"], np.float64)
    if len(orders) and any(cls[c][0] > 0 for c in cls):
        cls_of = psd_order_class(orders)
        dom = max((c for c in cls if cls[c][0] > 0), key=lambda c: cls[c][1])
        n_dom, ms_dom = cls[dom]
        flops = float(np.sum(EIG_FLOPS_PER_P3 * orders[cls_of == dom] ** 3))
        avg_ms = ms_dom / max(n_dom, 1)
        ach = flops / (avg_ms * 1e-3) / 1e12
        peak = PEAK_FP32_VECTOR_TFLOPS if wl["dtype"] == "f32" else PEAK_FP64_TFLOPS
        name = eig_kernel_name(dom, batch.psd_schedule()[0][dom], wl["dtype"] == "f32")
        rooflines["eig"] = {"kernel": name, "bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                            "frac": ach / peak,
                            "traffic": (traffic_from_profile(EIG_PROFILE, EIG_SOURCE, order_class=dom,
                                                             threads=batch.psd_schedule()[0][dom])
                                        if args.workload == "c2" else None),
                            "flops_per_launch": flops, "blocks_per_launch": int(np.sum(cls_of == dom)),
                            "avg_launch_ms": avg_ms, "launches": n_dom, "ms_per_step": ms_dom}
    n_pcg, ms_pcg = fam["pcg"]
    if n_pcg > 0:
        esz = 4 if wl["dtype"] == "f32" else 8
        gsz = 4 if wl.get("dense_f32") else esz
        iters = sprof["cg_iters_total"].astype(np.float64)
        passes = sprof["cg_passes_total"].astype(np.float64)
        # operator applications: one per iteration and one per float64 true-residual pass
        total = sum((iters[i] + passes[i]) * pcg_bytes_per_iteration(inst, esz, gsz)
                    for i, inst in enumerate(insts))
        avg_ms = ms_pcg / n_pcg
        ach = total / n_pcg / (avg_ms * 1e-3) / 1e9
        form = batch.pcg_form()
        tn = "float" if esz == 4 else "double"
        kname = (f"k_pcg_coop<{tn}> (cooperative, <= {form} workgroups per CU)" if form > 0
                 else f"k_pcg<{tn}> (one workgroup per instance"
                      + ((", dense blocks fused" + (", stored float32)" if gsz < esz else ")"))
                         if batch.n_dense else ")"))
        rooflines["pcg"] = {"kernel": kname, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": ach / PEAK_HBM_GBS,
                            "traffic": ({"c4": lambda: traffic_from_profile(PCG_PROFILE, PCG_SOURCE, pcg_form=form),
                                         "c5": lambda: traffic_from_profile(PCG_C5_PROFILE, PCG_SOURCE, pcg_form=form)}
                                        .get(args.workload, lambda: None)()),
                            "bytes_per_launch": total / n_pcg, "avg_launch_ms": avg_ms, "launches": n_pcg,
                            "mean_cg_iterations": float(iters.sum() / (n_pcg * B)),
                            "mean_residual_passes": float(passes.sum() / (n_pcg * B)),
                            "ms_per_step": ms_pcg}
    # the primary roofline is that of the kernel taking the most time per step
    primary = max(rooflines, key=lambda k: rooflines[k]["ms_per_step"]) if rooflines else None

    plain = None
    peak_plain = None
    if not args.no_plain:
        # the plain form: each instance alone, forward only, no tape, one
        # plan at a time (created, warmed up, timed, destroyed); its peak HBM
        # is the largest footprint of one such call (plan + buffers)
        del tape, fws, bws
        torch.cuda.empty_cache()
        n_plain = min(B, max(1, args.plain_sample))
        dt_plain, peak_plain = 0.0, 0
        for i in range(n_plain):
            torch.cuda.synchronize(dev)
            torch.cuda.reset_peak_memory_stats(dev)
            base_i = torch.cuda.memory_allocated(dev)
            free_i, res_i = torch.cuda.mem_get_info(dev)[0], torch.cuda.memory_reserved(dev)
            single = CosmoBatch([insts[i]], K=K, dtype=tdt, device=dev, **kw)
            torch.cuda.synchronize(dev)
            pb = max(0, (free_i - torch.cuda.mem_get_info(dev)[0]) - (torch.cuda.memory_reserved(dev) - res_i))
            srho = torch.from_numpy(rhos[i]).to(dev)
            salpha = torch.from_numpy(alphas[i].reshape(K, 1)).to(dev)
            single.forward(srho, salpha, tape=False)
            torch.cuda.synchronize(dev)
            t1 = time.perf_counter()
            single.forward(srho, salpha, tape=False)
            torch.cuda.synchronize(dev)
            dt_plain += time.perf_counter() - t1
            peak_plain = max(peak_plain, torch.cuda.max_memory_allocated(dev) - base_i + pb)
            single.close()
            del single, srho, salpha
        plain = {"value": n_plain * K / dt_plain, "unit": "instance-iterations/s", "ms_total": dt_plain * 1e3,
                 "instances": n_plain}
        print(f"[bench] plain forward {dt_plain * 1e3:.2f} ms for the first {n_plain} instances one by one",
              file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": B * K / dt,
        "unit": "instance-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl["dtype"],
        "data": "synthetic",
        "config": {"workload": wl["name"], "instances": B, "unroll_K": K,
                   "pass": "forward+loss+backward" if backward else "forward"},
        "peak_hbm_bytes": {"batched": int(peak_fb), "plain_fwd_one_instance": None if peak_plain is None
                           else int(peak_plain)},
        "plain_fwd": plain,
        "kernel_families_ms_per_step": {k: v[1] for k, v in fam.items()},
        "schedule": sched,
        "roofline": rooflines.get(primary),
        "roofline_other": {k: v for k, v in rooflines.items() if k != primary} or None,
        "stats": {k: int(v.max()) for k, v in batch.stats_dict(stats).items()},
    }

    if cpu is not None:
        wall, res, workers, n_s, steps = cpu
        out["cpu_baseline"] = {"value": n_s * steps / wall, "unit": "instance-iterations/s", "cores": workers,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"first {n_s} instances of the batch, first {steps} of {K} steps, "
                                         f"{'forward+loss+backward' if backward else 'forward'}, float64, "
                                         f"{workers} single-threaded processes"}
        # error of the timed GPU run against the oracle's full K-step runs:
        # the throughput sample when it covers all K steps, else the error leg
        ref_runs = None
        if steps == K:
            ref_runs = res
        elif err_leg is not None:
            (pool, pending), n_err = err_leg
            ref_runs = pending.get()
            pool.close()
            pool.join()
        if ref_runs is not None:
            per = []   # (iterate error, gradient error) per sampled instance
            xs, ss, ys = batch.split_n(fw.x), batch.split_m(fw.s), batch.split_m(fw.y)
            for i, (_, x, s, y, grho, galpha) in enumerate(ref_runs):
                e_it, e_g = 0.0, 0.0
                for gpu, ref in ((xs[i], x), (ss[i], s), (ys[i], y)):
                    e_it = max(e_it, np.linalg.norm(gpu.double().cpu().numpy() - ref) /
                               max(np.linalg.norm(ref), 1e-12))
                if backward:
                    gr = bw.grho[:, batch.m_off[i]:batch.m_off[i + 1]].double().cpu().numpy()
                    e_g = max(e_g, np.linalg.norm(gr - grho) / max(np.linalg.norm(grho), 1e-12))
                    ga = bw.galpha[:, i].double().cpu().numpy()
                    e_g = max(e_g, np.linalg.norm(ga - galpha) / max(np.linalg.norm(galpha), 1e-12))
                per.append((e_it, e_g))
            e_it = max(p[0] for p in per)
            e_g = max(p[1] for p in per)
            out["rel_err_vs_oracle"] = {"final_iterates_max": e_it, "gradients_max": e_g if backward else None,
                                        "instances": len(ref_runs), "steps": K}
            if wl["dtype"] == "f32" and not args.no_floor:
                # the float32 floor of the two sampled instances with the largest errors
                key = 1 if backward else 0
                worst = sorted(range(len(per)), key=lambda j: -per[j][key])[:2]
                f_it, f_g = float32_floor(wl, rhos, alphas, worst, [ref_runs[j] for j in worst])
                out["rel_err_vs_oracle"]["float32_floor"] = {
                    "instances": worst, "final_iterates_max": f_it, "gradients_max": f_g if backward else None,
                    "model": "the oracle with every stored per-step value rounded to float32 (nearest, and "
                             "two runs within one unit in the last place with solves stopped at the float32 "
                             "CG residual); largest error of the three against the exact run"}
                print(f"[bench] float32 floor on instances {worst}: iterates {f_it:.2e}, gradients {f_g:.2e}",
                      file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
