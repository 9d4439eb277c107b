"""Benchmark: regularised 3D solves per second at 256^3 to the discrepancy delta.

Workload (default): 128^3 grids on R and Y padded to 256^3, FP32 complex
transforms with FP64 kernel spectrum, norms and alpha search; each instance
has 5-10 Gaussian/box inclusions with amplitudes U[0.05, 0.8] and noise
delta in {1%, 3%, 5%}.  One step solves a batch of instances: for each,
set the data (forward transform), choose alpha by the discrepancy principle
(bisection in log10 alpha over [1e-8, 1]) and recover c.  Inputs are
synthesised on the GPU through the library's own forward operator before
the timed region and stay resident in HBM.

    python bench.py [--steps K] [--warmup W] [--batch B] [--n N] [--no-cpu]

Prints one JSON line.  Only the CPU-baseline leg calls the oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "regularized 3D solves/sec at 256^3 to discrepancy delta, learned-alpha vs bisection"
HBM_PEAK_GBS = 8000.0
PASS_NAMES = ["fwd_x", "fwd_y", "fwd_z", "inv_z", "inv_y", "inv_x"]


def pass_bytes(n, esz=4):
    """Algorithmic bytes of each pass for a cubic n^3 grid padded to P = 2n
    (reads of nonzero inputs + writes of kept outputs; complex = 2*esz)."""
    P = 2 * n
    kx = P // 2 + 1
    c = 2 * esz
    octant = kx * (P // 2 + 1) * (P // 2 + 1) * 16
    return {
        "fwd_x": n ** 3 * esz + kx * n * n * c,
        "fwd_y": kx * n * n * c + kx * n * P * c,
        "fwd_z": kx * n * P * c + kx * P * P * c,
        "inv_z": kx * P * P * c + octant + kx * n * P * 2 * c,
        "inv_y": kx * n * P * 2 * c + kx * n * n * 2 * c,
        "inv_x": kx * n * n * 2 * c + n ** 3 * esz,
    }


def make_instances(ctx, torch, n, batch, first_index=0):
    from paper_1703_01216_amd import inputs
    insts = []
    V0 = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    ctx.source_potential(V0, 1.0)
    for i in range(batch):
        inst = inputs.workload_instance(2, first_index + i, n=n)
        xi = torch.tensor(inst["xi"], dtype=torch.float32, device="cuda")
        zeta_true = xi * V0
        F = torch.empty_like(zeta_true)
        ctx.apply_operator(zeta_true, F)
        e = torch.tensor(inst["noise"], dtype=torch.float32, device="cuda")
        delta = ctx.add_noise(F, e, inst["delta_rel"])
        insts.append(dict(F=F, delta=delta, zeta=torch.empty_like(F), c=torch.empty_like(F),
                          delta_rel=inst["delta_rel"], index=first_index + i))
    return insts, V0


def cpu_baseline(n, mean_evals, n_sample_evals=3):
    """The oracle (numpy.fft FP64, as written) on one instance of the same workload."""
    import numpy as np

    from oracle import synth, tikhonov
    from oracle.geometry import Geom, sample_kernel
    from paper_1703_01216_amd import inputs

    g = Geom(n, n, n)
    inst = inputs.workload_instance(2, 0, n=n)
    d = synth.make_data(g, inst["xi"], inst["noise"], inst["delta_rel"])
    khat = np.fft.fftn(sample_kernel(g))
    t0 = time.perf_counter()
    for k in range(n_sample_evals):
        tikhonov.solve_spectral(g, khat, d["F"], 10.0 ** (-2 - k))
    dt = (time.perf_counter() - t0) / n_sample_evals
    value = 1.0 / (dt * mean_evals)
    return {"value": value, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sample_evals} oracle alpha evaluations (numpy.fft FP64, single thread) on one "
                      f"{n}^3 instance padded to {2 * n}^3, {dt:.2f} s each, scaled to the GPU's mean "
                      f"{mean_evals:.2f} evaluations per solve"}


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Plain device-to-device copy of a 1 GiB buffer (read + write = 2 GiB per
    copy): the practical HBM ceiling and the calibration kernel for counters."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes_per_copy": 2 * nbytes, "avg_us": ms * 1e3, "GB_s": 2 * nbytes / (ms * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the plain 1 GiB device copy used to calibrate traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1703_01216_amd import fr3d

    torch.cuda.set_device(0)
    copy = copy_bandwidth(torch)
    if args.copy_only:
        print(json.dumps({"copy": copy}))
        return
    n = args.n
    ctx = fr3d.Context(0)
    ctx.load_kernel(n, n, n, precision=32)
    insts, V0 = make_instances(ctx, torch, n, args.batch)
    print(f"[bench] {len(insts)} instances of {n}^3 ready", file=sys.stderr, flush=True)

    def step():
        evals = []
        for it in insts:
            ctx.set_data(it["F"], it["delta"])
            rep = ctx.solve_discrepancy(it["zeta"])
            ctx.recover_c(it["zeta"], V0, 1.0, it["c"])
            evals.append(rep["n_evals"])
            it["rep"] = rep
        return evals

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for p in range(6):
        ctx.get_timing(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = []
    for _ in range(args.steps):
        evals += step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = {PASS_NAMES[p]: ctx.get_timing(p) for p in range(6)}
    ctx.set_timing(False)
    elapsed = t1 - t0
    solves = args.steps * len(insts)
    value = solves / elapsed
    mean_evals = sum(evals) / len(evals)
    pb = pass_bytes(n)
    passes = {}
    for name, (ms, cnt) in timing.items():
        if cnt:
            avg = ms / cnt
            passes[name] = {"avg_us": avg * 1e3, "launches": cnt, "GB_s": pb[name] / (avg * 1e-3) / 1e9}
    dom = max(passes, key=lambda k: passes[k]["avg_us"] * passes[k]["launches"])
    ach = passes[dom]["GB_s"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_launch": pb[dom], "avg_launch_us": passes[dom]["avg_us"]}
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n}^3 grids padded to {2 * n}^3, batch {len(insts)} instances, "
                               f"5-10 inclusions, delta 1/3/5%, bisection to tol 1e-3",
                   "grid": n, "padded": 2 * n, "batch": len(insts), "search": "bisection",
                   "mean_evals_per_solve": mean_evals},
        "roofline": roofline,
        "passes": passes,
        "copy": copy,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, mean_evals)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
