"""Benchmark: shift x RHS solves per second of the shifted-COCG solver on one MI355X.

Default workload: the diamond tight-binding lattice of 8x8x8 conventional cells
(4096 atoms x 4 orbitals = 16384 rows, 278,528 stored entries), 256 shifts
eps in [-12, 8] with eta = 0.005, 256 unit right-hand sides e_0..e_255, every pair
solved to relative residual 1e-8 (iteration cap 40000), full solutions x_k,j written
to HBM.  A step is one complete solve of all 65,536 pairs with inputs resident on
the device.

Prints one JSON line with the metric, the roofline of the dominant kernel (the
deferred per-shift update, timed with HIP events on its stream) and the FP64 CPU
oracle timed on a bounded sample of the same workload.

Other workloads (--workload): `cubic` (16^3 lattice, 64 shifts, G_00 to 1e-10, the
latency-bound case) and `hubbard` (extended Hubbard ring, 11,778,624 rows, 128 shifts,
one complex right-hand side).  --variants prints, on stderr, the same diamond problem
at a reduced number of right-hand sides solved by the plain FP64 path (one rhs at a
time, shift vectors updated every iteration), by the blocked update, batched, and with
FP32 storage, with the error of each against the FP64 batched result.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
UPDATE_KERNEL_SOURCES = ["flush.hip", "device_common.h", "scocg_internal.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="diamond", choices=["diamond", "cubic", "hubbard"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--shifts-per-wg", type=int, default=0)
    ap.add_argument("--n-rhs", type=int, default=256)
    ap.add_argument("--n-shift", type=int, default=0)
    ap.add_argument("--max-iter", type=int, default=0)
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8000)
    ap.add_argument("--variants", type=int, default=0,
                    help="also compare solver forms on the diamond problem with this many rhs (stderr)")
    return ap.parse_args()


def update_kernel_digest():
    """sha1 over the sources the deferred-update kernel is compiled from."""
    import hashlib

    h = hashlib.sha1()
    for name in UPDATE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0802_0748_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of the update kernel from the committed rocprofv3 counter
    summary, if it was taken on this workload and the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"k_flush_{workload}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        digest = update_kernel_digest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha1") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(p, gpu_iters, sample_iters):
    """Time the oracle on one right-hand side with all shifts for a fixed number of
    iterations (and with a single shift, to separate the seed cost), then scale to
    the whole workload with the per-pair iteration counts of the GPU solve."""
    from oracle import oracle as O

    b = p.rhs_dense()[0]
    O.shifted_cocg(p.H, p.z[:1], b, fixed_iter=2)  # load / warm
    t0 = time.perf_counter()
    O.shifted_cocg(p.H, p.z, b, fixed_iter=sample_iters, seed_index=0)
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.shifted_cocg(p.H, p.z[:1], b, fixed_iter=sample_iters, seed_index=0)
    t_one = time.perf_counter() - t0
    M = len(p.z)
    c_seed = t_one / sample_iters
    c_pair = max(t_all - t_one, 0.0) / ((M - 1) * sample_iters)
    seed_iters = gpu_iters.max(axis=1).sum()
    est = c_seed * seed_iters + c_pair * gpu_iters.sum()
    converged = gpu_iters.size
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=converged / est, unit="solves/s", cores=threads, kind="oracle",
                sample=(f"oracle on the first rhs with all {M} shifts for {sample_iters} fixed iterations "
                        f"({t_all:.1f} s) and with one shift ({t_one:.1f} s); per-pair and per-seed iteration "
                        f"costs scaled by the GPU solve's iteration counts (sum {int(gpu_iters.sum())} pair-"
                        f"iterations, {int(seed_iters)} seed iterations) to an estimated {est:.0f} s"))


def load_workload(args):
    from workloads import config1_cubic, config2_diamond, config3_hubbard

    if args.workload == "diamond":
        p = config2_diamond(n_shift=args.n_shift or 256, n_rhs=args.n_rhs)
        p.max_iter, p.tol = 40000, 1e-8
        desc = (f"diamond 8x8x8 cells, 4 orbitals/atom (n={p.H.n}, nnz={p.H.nnz}), {len(p.z)} shifts eta=0.005, "
                f"{p.n_rhs} unit RHS")
    elif args.workload == "cubic":
        p = config1_cubic(n_shift=args.n_shift or 64)
        p.max_iter = 20000
        desc = f"simple cubic 16^3 (n={p.H.n}), {len(p.z)} shifts eta=0.01, G_00"
    else:
        p = config3_hubbard(n_shift=args.n_shift or 128)
        p.max_iter, p.tol = 20000, 1e-8
        desc = (f"extended Hubbard ring 14 sites 7+7 (n={p.H.n}, nnz={p.H.nnz}), {len(p.z)} shifts eta=0.05, "
                f"one complex unit RHS")
    if args.max_iter:
        p.max_iter = args.max_iter
    if args.tol:
        p.tol = args.tol
    return p, desc


def run_variants(S, torch, n_rhs):
    """The diamond problem with n_rhs right-hand sides solved by several forms of the solver."""
    from workloads import config2_diamond

    p = config2_diamond(n_rhs=n_rhs)
    H = S.Hamiltonian.from_csr(p.H)
    dev = torch.device("cuda")
    K, M, n = p.n_rhs, len(p.z), p.H.n
    B = torch.zeros((K, n), dtype=torch.complex128, device=dev)
    B[torch.arange(K), torch.from_numpy(p.rhs_idx).to(dev)] = 1.0
    base = dict(tol=1e-8, max_iter=40000)
    out = {}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    Xb, t_b = timed(lambda: S.shifted_cocg_solve(H, p.z, B, **base)[0])
    ref = Xb.cpu().numpy()
    out["batched fp64, block 24"] = (t_b, 0.0)
    forms = [("one rhs at a time, fp64, update every iteration (plain)", dict(block=1), 1),
             ("one rhs at a time, fp64, block 24", dict(block=24), 1),
             ("batched fp32 storage, block 24", dict(block=24, precision="fp32"), K),
             ("batched fp32 storage + fp64 refinement", dict(block=24, precision="fp32", refine=2), K)]
    for name, extra, per in forms:
        X = np.zeros_like(ref)
        t = 0.0
        for j0 in range(0, K, per):
            Xj, tj = timed(lambda: S.shifted_cocg_solve(H, p.z, B[j0:j0 + per], **base, **extra)[0])
            X[j0:j0 + per] = Xj.cpu().numpy()
            t += tj
        err = np.max(np.linalg.norm(X - ref, axis=2) / np.linalg.norm(ref, axis=2))
        out[name] = (t, err)
    print(f"[variants] diamond, {K} rhs x {M} shifts, tol 1e-8", file=sys.stderr)
    for name, (t, err) in out.items():
        print(f"[variants] {name:58s} {t:8.2f} s  {K * M / t:9.1f} solves/s  speedup vs plain "
              f"{out['one rhs at a time, fp64, update every iteration (plain)'][0] / t:6.2f}  max rel diff to "
              f"batched fp64 {err:.1e}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              "(the solver runs on a single device).", file=sys.stderr)
        return 2
    import torch

    import paper_0802_0748_amd as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p, desc = load_workload(args)
    H = S.Hamiltonian.from_csr(p.H)
    K, M, n = p.n_rhs, len(p.z), p.H.n
    greens = args.workload == "cubic"
    if not greens:
        B = torch.from_numpy(p.rhs_dense()).to(dev)
        X = torch.empty((K, M, n), dtype=torch.complex128, device=dev)
    opts = dict(tol=p.tol, max_iter=p.max_iter, precision=args.precision, block=args.block,
                shifts_per_wg=args.shifts_per_wg)

    def solve():
        if greens:
            return S.greens_diag(H, p.z, p.rhs_idx, **opts)
        return S.shifted_cocg_solve(H, p.z, B, out=X, **opts)

    print(f"[bench] workload {p.name}: n={n} nnz={p.H.nnz} shifts={M} rhs={K} {args.precision}", file=sys.stderr,
          flush=True)
    # initialise the library's code paths on a tiny problem (not a step)
    S.greens_diag(H, p.z[:4], p.rhs_idx[:1] if p.rhs_idx is not None else [0], fixed_iter=32, block=args.block,
                  precision=args.precision)
    torch.cuda.synchronize()
    S.set_profiling(True)
    for w in range(args.warmup):
        t0 = time.perf_counter()
        _, rep, _, rc = solve()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w}: {time.perf_counter() - t0:.2f} s rc={rc}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    upd_ms = upd_bytes = 0.0
    upd_launches = 0
    converged = 0
    iters = None
    t0 = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        _, rep, _, rc = solve()
        t = S.last_timing()
        upd_ms += t["update_ms"]
        upd_bytes += t["update_bytes"]
        upd_launches += t["update_launches"]
        converged += int((rep["status"] == 0).sum())
        iters = rep["iters"]
        print(f"[bench] step {s}: {time.perf_counter() - ts:.2f} s rc={rc} converged "
              f"{int((rep['status'] == 0).sum())}/{K * M} seed iterations {t['iterations']} "
              f"blocks {t['blocks']} switches {t['switches']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    S.set_profiling(False)
    value = converged / elapsed
    achieved = (upd_bytes / 1e9) / (upd_ms / 1e3) if upd_ms > 0 else 0.0
    line = {
        "metric": "shift x RHS solves/sec to rel. residual 1e-8",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-storage/f64-scalars",
        "data": "synthetic",
        "config": {"workload": f"{desc}, tol {p.tol:g}, max_iter {p.max_iter}",
                   "n": n, "nnz": int(p.H.nnz), "n_shift": M, "n_rhs": K, "precision": args.precision,
                   "block": args.block or 24, "iterations_per_step": int(np.max(iters))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload),
                     "kernel": "k_flush (deferred per-shift update)",
                     "avg_launch_ms": upd_ms / max(upd_launches, 1),
                     "bytes_per_launch": upd_bytes / max(upd_launches, 1)},
    }
    if not args.no_cpu_baseline:
        # the oracle's cost per iteration grows with shifts x rows: keep the sample near
        # --cpu-iters iterations of the diamond problem (256 x 16384)
        sample = max(10, min(100000, int(args.cpu_iters * 4194304 / (M * n))))
        line["cpu_baseline"] = cpu_baseline(p, iters, sample)
    if args.variants:
        run_variants(S, torch, args.variants)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
