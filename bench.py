"""Benchmark: batched forward + backward unrolled COSMO on one MI355X.

Workload (default): a batch of 64 max-cut SDPs, orders p ~ U{30..100}, edge
probability ~ U(0.1, 0.5), float32, K = 50 unrolled steps with per-step
penalties rho^k (per row) and relaxations alpha^k (per instance), loss =
final primal residual^2 + dual residual^2, backward to every rho^k, alpha^k.
One timed step = forward (K steps) + loss + backward (K steps) over the
whole batch, inputs resident in HBM.

Prints one JSON line: instance-iterations per second (B K / time per step),
peak HBM of the batched forward + backward against the plain forward
(unbatched, forward-only, no tape), the roofline of the dominant kernel
family measured with HIP events inside the library, the error against the
float64 oracle on a sample of instances, and the oracle's own throughput on
the host cores (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic work of one PSD block of order p: 9 p^3 for a textbook symmetric
# eigendecomposition (eigenvectors included) + 2 p^3 for U max(L, 0) U'.
EIG_FLOPS_PER_P3 = 11.0
# The library's PSD order classes and their float32 eigensolve kernels.
EIG_KERNEL_NAMES = {0: "k_psd_eig<float,64,4,32> (orders <= 32)", 1: "k_psd_eig<float,256,8,64> (orders 33-64)",
                    2: "k_psd_eig<float,512,8,128> (orders 65-128)", 3: "k_psd_eig<float,1024,8,200> (orders 129-200)"}
EIG_PROFILE = os.path.join(ROOT, "profiles", "k_psd_eig_maxcut64_pmc.md")
EIG_SOURCE = os.path.join(ROOT, "paper_2606_13825_amd", "csrc", "k_psd.hip")


def psd_order_class(orders):
    o = np.asarray(orders)
    return np.where(o <= 32, 0, np.where(o <= 64, 1, np.where(o <= 128, 2, 3)))


def traffic_from_profile(cls):
    """HBM bytes per dispatch of the class's eigensolve kernel, from the
    committed counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a copy kernel of known size); None when there is none for this
    class or the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        kv = {}
        with open(EIG_PROFILE) as f:
            for line in f:
                if ":" in line and line[:1].isalpha():
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        with open(EIG_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if kv.get("source_sha256") != sha or int(kv.get("order_class", -1)) != int(cls):
            return None
        return float(kv["traffic_bytes_per_dispatch"])
    except (OSError, KeyError, ValueError):
        return None


def _workload(name):
    import synth
    if name == "c2":
        insts = [x.astype(np.float32) for x in synth.c2_batch()]
        return dict(name="maxcut_sdp_batch64_p30-100_fp32_K50", insts=insts, K=50, dtype="f32", seed=2)
    raise SystemExit(f"unknown workload {name}")


def _hyper(insts, K, seed):
    import synth
    rng = np.random.default_rng(1000 + seed)
    rhos, alphas = [], []
    for inst in insts:
        r, a = synth.perturbed_hyper(inst, K, rng)
        rhos.append(r.astype(np.float32))
        alphas.append(a.astype(np.float32))
    return rhos, alphas


def _oracle_job(args):
    inst, rho, alpha = args
    import oracle
    t0 = time.perf_counter()
    tape, (x, s, y) = oracle.unroll_forward(inst, rho, alpha)
    g = oracle.residual_loss_grad(inst, x, s, y)
    grho, galpha, *_ = oracle.unroll_backward(inst, tape, *g)
    return time.perf_counter() - t0, x, s, y, grho, galpha


def cpu_baseline(insts, rhos, alphas, K, n_sample, workers):
    """The float64 oracle, as it stands, on the first n_sample instances,
    instance-parallel over `workers` single-threaded processes."""
    import multiprocessing as mp
    jobs = [(insts[i], rhos[i].astype(np.float64), alphas[i].astype(np.float64)) for i in range(n_sample)]
    # runs before this process touches the GPU, so forked workers are plain CPU processes
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_job, jobs)
    wall = time.perf_counter() - t0
    return wall, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB five times (reference for the HBM byte counters)")
    ap.add_argument("--quick", action="store_true",
                    help="counter-collection run: the timed steps only (no plain-forward comparison, "
                         "no event-timed step, no CPU leg)")
    args = ap.parse_args()
    if args.quick:
        args.no_cpu_baseline = True
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU: the batch shards over instances with no "
                                   "exchange inside the unroll, but runs on more than one GPU are not part of it"}))
        raise SystemExit(2)

    if args.copy_calibration:
        import torch
        n = 64 * 1024 * 1024
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "dispatches": 5}))
        return

    wl = _workload(args.workload)
    insts, K = wl["insts"], wl["K"]
    B = len(insts)
    rhos, alphas = _hyper(insts, K, wl["seed"])
    print(f"[bench] workload {wl['name']}: B={B} K={K}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        try:
            aff = len(os.sched_getaffinity(0))
        except AttributeError:
            aff = os.cpu_count() or 1
        workers = max(1, min(16, aff, args.cpu_sample))
        n_s = min(args.cpu_sample, B)
        wall, res = cpu_baseline(insts, rhos, alphas, K, n_s, workers)
        cpu = (wall, res, workers, n_s)
        print(f"[bench] cpu baseline: {n_s} instances in {wall:.1f} s on {workers} processes", file=sys.stderr,
              flush=True)

    import torch
    from paper_2606_13825_amd import CosmoBatch

    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)          # initialise the device before the memory counters

    torch.cuda.reset_peak_memory_stats(dev)
    base_mem = torch.cuda.memory_allocated(dev)
    batch = CosmoBatch(insts, K=K, dtype=torch.float32, device=dev)
    rho = torch.from_numpy(np.concatenate(rhos, axis=1)).to(dev)
    alpha = torch.from_numpy(np.stack(alphas, axis=1)).to(dev)
    tape = batch.new_tape()
    fws, bws = batch.new_fwd_ws(), batch.new_bwd_ws()
    stats = batch.new_stats()

    def step():
        fw = batch.forward(rho, alpha, tape=tape, ws=fws, stats=stats)
        loss, g = batch.residual_loss(fw.x, fw.s, fw.y, ws=fws)
        bw = batch.backward(rho, alpha, fw.tape, *g, ws=bws, stats=stats)
        return fw, loss, bw

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fw, loss, bw = step()
    torch.cuda.synchronize(dev)
    dt = (time.perf_counter() - t0) / args.steps
    peak_fb = torch.cuda.max_memory_allocated(dev) - base_mem
    print(f"[bench] fwd+bwd {dt * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    if args.quick:
        print(json.dumps({"metric": "fwd+bwd unrolled COSMO iters/s (counter-collection run)",
                          "value": B * K / dt, "unit": "instance-iterations/s", "ms_per_step": dt * 1e3}))
        return

    # kernel families, and the eigensolve kernel of each PSD order class alone,
    # timed with HIP events recorded by the library on the streams they run on
    batch.set_profiling(True)
    step()
    torch.cuda.synchronize(dev)
    fam = {}
    for kind, name in ((0, "psd_eig_project"), (1, "psd_dk_vjp"), (2, "pcg"), (3, "csr_row_col_passes")):
        fam[name] = batch.profile_read(kind)
    cls = {c: batch.profile_read(4 + c) for c in range(4)}
    batch.set_profiling(False)
    orders = np.array([inst.meta["order"] for inst in insts], np.float64)
    cls_of = psd_order_class(orders)
    dom = max((c for c in cls if cls[c][0] > 0), key=lambda c: cls[c][1])
    n_dom, ms_dom = cls[dom]
    dom_flops = float(np.sum(EIG_FLOPS_PER_P3 * orders[cls_of == dom] ** 3))
    avg_dom_ms = ms_dom / max(n_dom, 1)
    achieved = dom_flops / (avg_dom_ms * 1e-3) / 1e12
    print(f"[bench] kernel families (launches, ms): {fam}", file=sys.stderr, flush=True)
    print(f"[bench] eigensolve per order class (launches, ms): {cls}", file=sys.stderr, flush=True)

    # plain forward: unbatched, forward-only, no tape
    del tape, fws, bws
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)
    base_mem2 = torch.cuda.memory_allocated(dev)
    singles = [CosmoBatch([inst], K=K, dtype=torch.float32, device=dev) for inst in insts]
    srho = [torch.from_numpy(r).to(dev) for r in rhos]
    salpha = [torch.from_numpy(a.reshape(K, 1)).to(dev) for a in alphas]
    for i in range(min(2, B)):
        singles[i].forward(srho[i], salpha[i], tape=False)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    for i in range(B):
        singles[i].forward(srho[i], salpha[i], tape=False)
    torch.cuda.synchronize(dev)
    dt_plain = time.perf_counter() - t1
    peak_plain = torch.cuda.max_memory_allocated(dev) - base_mem2
    print(f"[bench] plain forward {dt_plain * 1e3:.2f} ms for B={B}", file=sys.stderr, flush=True)

    out = {
        "metric": "fwd+bwd unrolled COSMO iters/s & peak HBM vs plain fwd, at 1e-5 rel err",
        "value": B * K / dt,
        "unit": "instance-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "instances": B, "unroll_K": K, "pass": "forward+loss+backward",
                   "psd_orders": [int(o) for o in orders]},
        "peak_hbm_bytes": {"fwd_bwd_batched": int(peak_fb), "plain_fwd_unbatched": int(peak_plain)},
        "plain_fwd": {"value": B * K / dt_plain, "unit": "instance-iterations/s", "ms_total": dt_plain * 1e3},
        "kernel_families_ms_per_step": {k: v[1] for k, v in fam.items()},
        "roofline": {"kernel": EIG_KERNEL_NAMES[dom], "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": traffic_from_profile(dom),
                     "flops_per_launch": dom_flops, "blocks_per_launch": int(np.sum(cls_of == dom)),
                     "avg_launch_ms": avg_dom_ms, "launches": n_dom},
        "stats": {k: int(v.max()) for k, v in batch.stats_dict(stats).items()},
    }

    if cpu is not None:
        wall, res, workers, n_s = cpu
        out["cpu_baseline"] = {"value": n_s * K / wall, "unit": "instance-iterations/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"first {n_s} instances of the batch, forward+loss+backward, K={K}, "
                                         f"float64, {workers} single-threaded processes"}
        # error of the timed GPU run against the oracle on the same sample
        e_it, e_g = 0.0, 0.0
        xs, ss, ys = batch.split_n(fw.x), batch.split_m(fw.s), batch.split_m(fw.y)
        for i, (_, x, s, y, grho, galpha) in enumerate(res):
            for gpu, ref in ((xs[i], x), (ss[i], s), (ys[i], y)):
                e_it = max(e_it, np.linalg.norm(gpu.double().cpu().numpy() - ref) / max(np.linalg.norm(ref), 1e-12))
            gr = bw.grho[:, batch.m_off[i]:batch.m_off[i + 1]].double().cpu().numpy()
            e_g = max(e_g, np.linalg.norm(gr - grho) / max(np.linalg.norm(grho), 1e-12))
            ga = bw.galpha[:, i].double().cpu().numpy()
            e_g = max(e_g, np.linalg.norm(ga - galpha) / max(np.linalg.norm(galpha), 1e-12))
        out["rel_err_vs_oracle"] = {"final_iterates_max": e_it, "gradients_max": e_g, "instances": n_s}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
