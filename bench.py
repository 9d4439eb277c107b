"""Benchmark: regularised 3D solves per second at 256^3 to the discrepancy delta,
learned alpha vs bisection.

Workload: 128^3 grids on R and Y padded to 256^3 (default gap D = 160 cells),
FP32 complex transforms with the FP64 kernel spectrum, norms and alpha search.
A batch of instances with 5-10 Gaussian/box inclusions of amplitude
U[0.05, 0.8] and noise delta cycling through 1%, 3%, 5% is synthesised on
the GPU through the library's own forward operator before any timing and
stays resident in HBM.  One step solves the whole batch with the lane
scheduler: per instance the forward transform of F, the alpha search and the
recovery of c.

Searches run on the same batch (config.modes):
  learned      -- the predictor fine-tuned on the GPU for this geometry on
                  untimed instances (calibrate.fine_tune), its seed refined by
                  secant steps on ln(r/T) whose first step assumes the
                  calibrated median slope (a seed next to the lower range end
                  starts there); every point accepted when |r/delta - 1| <=
                  1e-3 (the headline value)
  learned_ratio -- the same with the first step's slope taken from the
                  whole-box residual at the seed (formed by the seed's own
                  evaluation) times the calibrated ratio
  bisection    -- plain bisection over log10 alpha in [-8, 0] to |r/delta - 1| <= 1e-3
  learned_net  -- the shipped network alone (no fine-tuning), secant steps with
                  the median root slope of its training instances
  learned_w, bisection_w -- the learned and bisection searches with the wider
                  acceptance |r/delta - 1| <= 0.1
  kary16       -- the 16-candidate search
Then single-lane sections time every pass kernel with HIP events at 256^3
(the roofline of the dominant kernel) and at 512^3 (roofline_512: volumes
far beyond the last-level cache), the batch is solved in FP64 too, the
exact-operator CG solve, the uneven-size batch and the per-frequency form
are timed once each, and the CPU oracle is timed on whole solves of the
first instances (one process and 16 processes) beside per-result precision
checks of the device's estimates against it.

    python bench.py [--steps K] [--warmup W] [--batch B] [--n N] [--lanes L] [--modes M,...]
                    [--calibrate C] [--graphs 0|1] [--no-cpu] [--roofline-only]

Prints one JSON line.  Only the CPU-baseline leg calls the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "regularized 3D solves/sec at 256^3 to discrepancy delta, learned-alpha vs bisection"
HBM_PEAK_GBS = 8000.0
CAL_FIRST = 100000  # first instance index of the seed calibration set (disjoint from the timed batch)
PASS_NAMES = ["fwd_x", "fwd_y", "fwd_z", "inv_z", "inv_y", "inv_x"]
# HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE (scaled by the
# plain-copy calibration factors 2.000 and 1.000), valid only for the pass
# sources with this digest and the tile codes they were taken with; see
# profiles/passes_256cube_traffic.md and profiles/passes_512cube_traffic.md.
MEASURED_TRAFFIC = {"digest": "05ee041c09fd10ab", "n": 128,
                    "tiles": {"fwd_x": 0, "fwd_y": 1, "fwd_z": 0, "inv_x": 0, "inv_y": 1, "inv_z": 0},
                    "bytes": {"inv_z": 152.9e6, "inv_y": 101.5e6, "inv_x": 42.4e6, "fwd_z": 111.1e6,
                              "fwd_y": 50.8e6, "fwd_x": 25.4e6}}
MEASURED_TRAFFIC_512 = {"digest": "05ee041c09fd10ab", "n": 256,
                        "tiles": {"fwd_x": 0, "fwd_y": 9, "fwd_z": 0, "inv_x": 8, "inv_y": 9, "inv_z": 0},
                        "bytes": {"inv_z": 1216.8e6, "inv_y": 808.6e6, "inv_x": 337.0e6, "fwd_z": 884.1e6,
                                  "fwd_y": 404.4e6, "fwd_x": 202.0e6}}


def pass_source_digest():
    import hashlib
    d = os.path.join(ROOT, "paper_1703_01216_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read()
                   for f in ("fft_core.hpp", "passes.hpp", "passes_impl.hpp", "control.hpp"))
    return hashlib.sha256(src).hexdigest()[:16]


def pass_bytes(n, esz=4, shape=None):
    """Algorithmic bytes of each pass for an n^3 grid (or shape = (nz, ny, nx))
    padded to P = 2n per axis: reads of the nonzero inputs plus writes of the
    kept outputs (complex = 2 esz; the Tikhonov filter reads the kernel
    spectrum's octant as complex of the same precision: the FP32 path its
    FP32 rounding, the FP64 path the FP64 octant; the forward z pass reads
    the octant's byte table of kernel-spectrum levels for the features)."""
    nz, ny, nx = shape or (n, n, n)
    Pz, Py = 2 * nz, 2 * ny
    kx = nx + 1
    c = 2 * esz
    cells = nx * ny * nz
    octant = kx * (Pz // 2 + 1) * (Py // 2 + 1) * c
    levels = kx * (Py // 2 + 1) * Pz  # byte table of kernel-spectrum levels, rows over all kz
    return {
        "fwd_x": cells * esz + kx * nz * ny * c,
        "fwd_y": kx * nz * ny * c + kx * nz * Py * c,
        "fwd_z": kx * nz * Py * c + kx * Pz * Py * c + levels,
        "inv_z": kx * Pz * Py * c + octant + kx * nz * Py * 2 * c,
        "inv_y": kx * nz * Py * 2 * c + kx * nz * ny * 2 * c,
        "inv_x": kx * nz * ny * 2 * c + cells * esz,
    }


def make_instances(ctx, torch, n, batch, first=0):
    from paper_1703_01216_amd import inputs
    V0 = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    ctx.source_potential(V0, 1.0)
    Fs, deltas = [], []
    for i in range(first, first + batch):
        seed = inputs.instance_seed(2, i)
        xi = inputs.xi_torch((n, n, n), inputs.inclusion_params((n, n, n), seed))
        F = torch.empty_like(xi)
        ctx.apply_operator(xi * V0, F)
        e = inputs.noise_torch((n, n, n), seed)
        deltas.append(ctx.add_noise(F, e, (0.01, 0.03, 0.05)[i % 3]))
        Fs.append(F)
    return Fs, deltas, V0


def _oracle_task(task):
    """Work of one oracle process (spawned, so it holds no GPU state).
    kind "solve": one whole discrepancy solve of an instance by the oracle as
    written (numpy.fft FP64, three transforms per alpha evaluation), either
    the plain bisection rule or the learned search (features, the network in
    FP64 with BF16-rounded operands, the seeded secant rule); the kernel
    spectrum is set-up and not timed.  kind "check": the oracle's estimate
    at the device's alpha against the device's zeta (relative L2) and the
    oracle's r/delta there."""
    import numpy as np

    from oracle import discrepancy, features, mlp, tikhonov
    from oracle.geometry import Geom, sample_kernel
    from oracle.operator import pad

    F, delta = task["F"], task["delta"]
    nz, ny, nx = F.shape
    g = Geom(nx, ny, nz)
    khat = np.fft.fftn(sample_kernel(g))
    if task["kind"] == "check":
        o = tikhonov.solve_spectral(g, khat, F, task["alpha"])
        z = task["zeta"]
        return {"rel_l2": float(np.linalg.norm(z - o["zeta"]) / np.linalg.norm(o["zeta"])),
                "oracle_r_over_delta": o["r_norm"] / delta, "device_r_over_delta": task["residual"] / delta}

    def ev(a):
        o = tikhonov.solve_spectral(g, khat, F, a)
        return o["r_norm"], o["zeta_norm"]

    t0 = time.perf_counter()
    if task["mode"] == "bisection":
        res = discrepancy.bisection(ev, delta, tol=1e-3)
    else:
        params, norm, opts = task["net"]
        s = (khat * khat.conj()).real
        x, _ = features.features(np.fft.fftn(pad(g, F)), delta, float(np.linalg.norm(F)), s, float(s.max()))
        p, k = {}, 0
        for name, shape in mlp.PARAM_SHAPES:
            m = int(np.prod(shape))
            p[name] = np.asarray(params[k:k + m], dtype=np.float64).reshape(shape)
            k += m
        xs = (x - norm[:65]) / norm[65:130]
        y, _ = mlp.forward(p, xs[None, :], bf16=True)
        t_seed = float(norm[130] + norm[131] * y[0])
        res = discrepancy.seeded_secant(ev, delta, t_seed, tol=1e-3, acc_lo=1 - 1e-3, acc_hi=1 + 1e-3,
                                        slope=opts["seed_slope"], snap=opts.get("seed_snap_lo", 0.0),
                                        slope_ratio=opts.get("seed_slope_ratio", 0.0),
                                        slope_at=lambda t: tikhonov.full_box_slope(g, khat, F, 10.0 ** t))
    return {"seconds": time.perf_counter() - t0, "n_evals": res["n_evals"], "alpha": res["alpha"],
            "flags": res["flags"]}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(Fh, deltas, net, checks, workers=16):
    """The oracle timed on the host: whole solves (not extrapolated) of the
    first instances of the timed batch, the learned search (the headline's
    network and options) and bisection, on one process and on `workers`
    processes at once (one solve each; numpy's transforms are single-threaded,
    so a process is a core), and the per-result precision checks of the
    device's estimates."""
    import multiprocessing as mp

    workers = max(1, min(workers, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    out = {"cores": workers, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    # one thread per process (the workers inherit this environment when spawned)
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    os.environ.update({k: "1" for k in keep})
    try:
        return _cpu_pool(out, ctx, workers, Fh, deltas, net, checks)
    finally:
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _cpu_pool(out, ctx, workers, Fh, deltas, net, checks):
    import concurrent.futures as cf
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        list(ex.map(_oracle_task, [{"kind": "check", "F": Fh[0][:8, :8, :8].copy(), "delta": 1.0, "alpha": 1.0,
                                    "zeta": Fh[0][:8, :8, :8].copy(), "residual": 1.0}] * workers))  # warm the pool
        for mode in (("learned", "bisection") if net is not None else ("bisection",)):
            one = _oracle_task({"kind": "solve", "mode": mode, "F": Fh[0], "delta": deltas[0], "net": net})
            tasks = [{"kind": "solve", "mode": mode, "F": Fh[i % len(Fh)], "delta": deltas[i % len(Fh)], "net": net}
                     for i in range(workers)]
            t0 = time.perf_counter()
            res = list(ex.map(_oracle_task, tasks))
            wall = time.perf_counter() - t0
            out[mode] = {"solves_per_s_1_core": 1.0 / one["seconds"], "seconds_1_core": one["seconds"],
                         "n_evals_1_core": one["n_evals"],
                         f"solves_per_s_{workers}_cores": workers / wall, "wall_s": wall,
                         "mean_evals": sum(r["n_evals"] for r in res) / len(res)}
        out["precision_checks"] = list(ex.map(_oracle_task, checks))
    mode = "learned" if net is not None else "bisection"
    L = out[mode]
    out.update({"value": L[f"solves_per_s_{workers}_cores"], "unit": "solves/s", "kind": "oracle",
                "sample": f"whole oracle solves (numpy.fft FP64, the {mode} search with the headline's network "
                          f"and options) of the first {workers} instances of the timed batch, one per process on "
                          f"{workers} processes at once ({L['wall_s']:.1f} s wall); one process alone: "
                          f"{L['seconds_1_core']:.1f} s per solve"})
    return out


def workload3_section(torch, fr3d, n_inst=64, steps=2, warmup=1, graphs=(False, True), modes=("kary16", "bisection")):
    """Batched solves of the uneven-size workload: n_inst instances (each axis
    from {64, 96, 128, 192}), each under the four source sets q (one context
    and stream per (instance, q)), all scheduled together by the group solver
    (the 16-candidate search borrows its workspaces from a pool of a few
    slots); the 16-candidate search and bisection, both to 1e-3, with and
    without the lanes' evaluations replayed as HIP graphs.  Then the latency of
    one solve alone (one context, one lane) with each search, per grid size."""
    from paper_1703_01216_amd import inputs
    tight = dict(tol=1e-3, accept_lo=1 - 1e-3, accept_hi=1 + 1e-3)
    ctxs, Fs, deltas, shapes = [], [], [], []
    t0 = time.perf_counter()
    for i in range(n_inst):
        r = inputs.workload_params(3, i)
        shape = r["shape"]
        nz, ny, nx = shape
        for q in r["q"]:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                c = fr3d.Context(0, stream=st)
                c.load_kernel(nx, ny, nz, q=q, precision=32)
                c.apply_tuning(batched=True)
                V = torch.empty(shape, dtype=torch.float32, device="cuda")
                c.source_potential(V)
                xi = inputs.xi_torch(shape, r["inclusions"])
                F = torch.empty_like(xi)
                c.apply_operator(xi * V, F)
                e = inputs.noise_torch(shape, r["seed"])
                deltas.append(c.add_noise(F, e, r["delta_rel"]))
            ctxs.append(c)
            Fs.append(F)
            shapes.append(shape)
    torch.cuda.synchronize()
    cells = sum(s[0] * s[1] * s[2] for s in shapes)
    out = {"instances": n_inst, "items": len(Fs), "distinct_shapes": len(set(shapes)),
           "setup_s": time.perf_counter() - t0, "cells_per_item_mean": cells / len(Fs)}
    zs = [torch.empty_like(F) for F in Fs]
    for m in modes:
        o = fr3d.default_opts(candidates=int(m[4:]), **tight) if m.startswith("kary") else fr3d.default_opts(**tight)
        for gr in graphs:
            for c in ctxs:
                c.set_graphs(gr)
            for _ in range(warmup):
                fr3d.solve_group(ctxs, Fs, deltas, zs, opts=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            evals = []
            for _ in range(steps):
                reps = fr3d.solve_group(ctxs, Fs, deltas, zs, opts=o)
                evals += [r["n_evals"] for r in reps]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            row = {"solves_per_s": len(Fs) * steps / el, "mean_evals": sum(evals) / len(evals),
                   "alpha_evals_per_s": sum(evals) / el, "ms_per_step": el / steps * 1e3}
            if not m.startswith("kary"):
                # algorithmic bytes of the forward transform, the evaluations and
                # the recovery of every item over the time
                tot = 0
                for k, shp in enumerate(shapes):
                    pb = pass_bytes(0, shape=shp)
                    tot += sum(pb[p] for p in ("fwd_x", "fwd_y", "fwd_z"))
                    tot += evals[k] * sum(pb[p] for p in ("inv_z", "inv_y", "inv_x"))
                row["aggregate_GB_s"] = tot * steps / el / 1e9
            out[f"{m}{'_graphs' if gr else ''}"] = row
    for c in ctxs:
        c.set_graphs(False)
    # latency of a single solve, per grid size (the first item of each cubic-ish size)
    lat = {}
    for n in (64, 128, 192):
        k = next((i for i, s in enumerate(shapes) if max(s) == n and min(s) == n), None)
        if k is None:
            k = next((i for i, s in enumerate(shapes) if max(s) == n), None)
        if k is None:
            continue
        row = {"shape": list(shapes[k])}
        c = ctxs[k]
        for m in modes:
            o = fr3d.default_opts(candidates=int(m[4:]), **tight) if m.startswith("kary") else fr3d.default_opts(**tight)
            c.set_data(Fs[k], deltas[k])
            c.solve_discrepancy(zs[k], opts=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                c.set_data(Fs[k], deltas[k])
                rep = c.solve_discrepancy(zs[k], opts=o)
            torch.cuda.synchronize()
            row[m] = {"ms": (time.perf_counter() - t0) / 5 * 1e3, "n_evals": rep["n_evals"]}
        lat[f"max_axis_{n}"] = row
    # small cubic grids, where an evaluation cannot fill the GPU
    for n in (32, 64):
        shape = (n, n, n)
        c = fr3d.Context(0)
        c.load_kernel(n, n, n, q=0, precision=32)
        c.apply_tuning()
        V = torch.empty(shape, dtype=torch.float32, device="cuda")
        c.source_potential(V)
        r = inputs.workload_params(3, 0)
        xi = inputs.xi_torch(shape, inputs.inclusion_params(shape, r["seed"]))
        F = torch.empty_like(xi)
        c.apply_operator(xi * V, F)
        dl = c.add_noise(F, inputs.noise_torch(shape, r["seed"]), 0.02)
        z = torch.empty_like(F)
        row = {"shape": list(shape)}
        for m in modes:
            o = fr3d.default_opts(candidates=int(m[4:]), **tight) if m.startswith("kary") else fr3d.default_opts(**tight)
            c.set_data(F, dl)
            c.solve_discrepancy(z, opts=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                c.set_data(F, dl)
                rep = c.solve_discrepancy(z, opts=o)
            torch.cuda.synchronize()
            row[m] = {"ms": (time.perf_counter() - t0) / 10 * 1e3, "n_evals": rep["n_evals"]}
        lat[f"cube_{n}"] = row
        c.close()
    out["single_solve_latency"] = lat
    for c in ctxs:
        c.close()
    return out


def layered_section(torch, fr3d, n=256, nz=51, reps=3):
    """Algorithm 1 with per-frequency z-systems at the size the paper times
    (Sec. 6: lateral grid N = 512, M = M' = 51 layers): n x n x nz cells, the
    lateral axes padded to 2n = 512.  Times the setup (lateral kernel
    transform + one SVD per distinct system) and whole solves (data
    transform, discrepancy search to 1e-3 over alpha in [1e-12, 1], inverse)
    with TSVD -- the paper's best method -- and with Tikhonov; 5% noise."""
    from paper_1703_01216_amd import inputs
    shape = (nz, n, n)
    c = fr3d.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.load_layered(n, n, nz, precision=32)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    V = torch.empty(shape, dtype=torch.float32, device="cuda")
    c.source_potential(V)
    seed = inputs.instance_seed(2, 0)
    xi = inputs.xi_torch(shape, inputs.inclusion_params(shape, seed))
    F = torch.empty_like(xi)
    c.apply_operator(xi * V, F)
    delta = c.add_noise(F, inputs.noise_torch(shape, seed), 0.05)
    z = torch.empty_like(F)
    out = {"grid": list(shape), "lateral_padded": 2 * n, "setup_ms": setup * 1e3,
           "paper": "MATLAB, one core: N = 512, M = M' = 51 solved in under 10 minutes (Sec. 6)"}
    for name, (kind, order) in (("tsvd", (2, 1)), ("tikhonov", (0, 1))):
        c.set_filter(kind, order)
        c.set_data(F, delta)
        c.solve_discrepancy(z, tol=1e-3, log10_alpha_lo=-12.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c.set_data(F, delta)
            rep = c.solve_discrepancy(z, tol=1e-3, log10_alpha_lo=-12.0)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        out[name] = {"solve_ms": el * 1e3, "n_evals": rep["n_evals"], "flags": rep["flags"],
                     "alpha": rep["alpha"], "r_over_delta": rep["residual"] / delta}
        # Algorithm 1 step 2 per lateral frequency: every system's own alpha
        # (bisection on its closed-form residual), then one lateral inverse
        c.solve_per_frequency(z, tol=1e-3, log10_alpha_lo=-12.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c.set_data(F, delta)
            rep = c.solve_per_frequency(z, tol=1e-3, log10_alpha_lo=-12.0)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        out[name + "_per_frequency"] = {"solve_ms": el * 1e3, "flags": rep["flags"],
                                        "mean_alpha": rep["alpha"], "r_over_delta": rep["residual"] / delta}
    c.close()
    # the model example itself (Sec. 6 geometry and xi, FP64, TSVD, perturbation 1e-3)
    from paper_1703_01216_amd import model_example
    me = model_example.run(n, nz, amplitude=1e-3, precision=64)
    out["model_example_fp64_tsvd"] = {k: me[k] for k in ("setup_ms", "solve_ms", "n_evals", "flags", "alpha",
                                                           "r_over_delta", "singular_values")}
    out["model_example_fp64_tsvd"]["mean_delta_C"] = sum(me["delta_C"]) / len(me["delta_C"])
    return out


def exact_section(torch, fr3d, Fs, n, alpha=1e-3, max_iter=200):
    """Tikhonov for the exact restricted operator (CG on the normal
    equations, two transform round trips per step) on one instance of the
    bench workload: per-step time and the estimate's gap to the 3D
    embedding's at the same alpha."""
    c = fr3d.Context(0)
    c.load_kernel(n, n, n, precision=32)
    c.apply_tuning()
    F = Fs[0]
    z = torch.empty_like(F)
    c.solve_exact(F, alpha, z, max_iter=2, tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = c.solve_exact(F, alpha, z, max_iter=max_iter, tol=1e-6)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ze = torch.empty_like(F)
    c.set_data(F, 1.0)
    re = c.solve_alpha(alpha, ze)
    gap = float(torch.linalg.vector_norm((z - ze).double()) / torch.linalg.vector_norm(ze.double()))
    c.close()
    return {"alpha": alpha, "cg_steps": rep["n_evals"], "converged": rep["flags"] == 0,
            "ms_per_cg_step": el / max(rep["n_evals"], 1) * 1e3, "solve_ms": el * 1e3,
            "residual_exact": rep["residual"], "residual_embedded": re["residual"],
            "zeta_gap_to_embedded": gap}


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


def copy_sweep(torch, reps=20):
    """Plain device copies that move as many bytes as each pass kernel does
    at 128^3 -> 256^3 and 256^3 -> 512^3 (half read, half written): the
    practical ceiling of a kernel of that size, launch and drain included.
    Timed by events around `reps` back-to-back copies (the kernel trace of the
    same run gives the per-kernel durations)."""
    out = {}
    for n in (128, 256):
        for name, b in pass_bytes(n).items():
            half = b // 2 // 4
            src = torch.empty(half, dtype=torch.float32, device="cuda").fill_(1.0)
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                dst.copy_(src)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            out[f"{2 * n}^3 {name}"] = {"bytes": 2 * half * 4, "avg_us": us, "GB_s": 2 * half * 4 / (us * 1e-6) / 1e9}
            del src, dst
    return out


def kernel_timing(ctx, torch, Fs, deltas, opts, lanes):
    """Per-pass kernel durations from HIP events recorded at each pass
    kernel's start and end, on one lane so that no two pass kernels overlap:
    the bisection search to 1e-3 over the whole batch."""
    ctx.set_lanes(1)
    zs = [torch.empty_like(F) for F in Fs]
    ctx.solve_batch(Fs[:2], deltas[:2], zs[:2], opts=opts)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for p in range(6):
        ctx.get_timing(p)
    t0 = time.perf_counter()
    ctx.solve_batch(Fs, deltas, zs, opts=opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = {PASS_NAMES[p]: ctx.get_timing(p) for p in range(6)}
    ctx.set_timing(False)
    ctx.set_lanes(lanes)
    return tm, el


def pass_table(timing, pb):
    passes = {}
    for name, (ms, cnt) in timing.items():
        if cnt:
            avg = ms / cnt
            passes[name] = {"avg_us": avg * 1e3, "launches": cnt, "GB_s": pb[name] / (avg * 1e-3) / 1e9,
                            "frac": pb[name] / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, "total_ms": ms}
    return passes


def roofline_of(passes, pb, traffic_table, n, tiles):
    dom = max(passes, key=lambda k: passes[k]["total_ms"])
    ach = passes[dom]["GB_s"]
    traffic = None
    # the counters hold for the kernels they were taken on: same sources, size and tile codes
    if (traffic_table and pass_source_digest() == traffic_table["digest"] and n == traffic_table["n"]
            and (tiles or {}).get(dom) == traffic_table["tiles"].get(dom)):
        traffic = traffic_table["bytes"].get(dom)
    return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": pb[dom],
            "avg_launch_us": passes[dom]["avg_us"], "tile_code": (tiles or {}).get(dom)}


def section_512(torch, fr3d, reps=8, alpha=1e-6):
    """Single-lane pass timing at the precision-stress size, 256^3 grids
    padded to 512^3 (FP32 complex volumes of 1 GiB: far beyond the 256 MB
    last-level cache, so every pass streams from HBM): one workload-4
    instance synthesised on the device, then `reps` forward transforms and
    `reps` evaluations at a fixed alpha, each pass kernel timed with HIP
    events at its own start and end."""
    from paper_1703_01216_amd import inputs
    n = 256
    shape = (n, n, n)
    c = fr3d.Context(0)
    c.load_kernel(n, n, n, precision=32)
    tuning = c.apply_tuning()
    inst = inputs.workload_instance(4, 0)
    V0 = torch.empty(shape, dtype=torch.float32, device="cuda")
    c.source_potential(V0)
    xi = torch.tensor(inst["xi"], dtype=torch.float32, device="cuda")
    F = torch.empty_like(xi)
    c.apply_operator(xi * V0, F)
    delta = c.add_noise(F, torch.tensor(inst["noise"], dtype=torch.float32, device="cuda"), inst["delta_rel"])
    del xi
    z = torch.empty_like(F)
    c.set_data(F, delta)
    c.solve_alpha(alpha, z)
    torch.cuda.synchronize()
    c.set_timing(True)
    for p in range(6):
        c.get_timing(p)
    for _ in range(reps):
        c.set_data(F, delta)
        c.solve_alpha(alpha, z)
    torch.cuda.synchronize()
    timing = {PASS_NAMES[p]: c.get_timing(p) for p in range(6)}
    c.set_timing(False)
    c.close()
    del F, z, V0
    torch.cuda.empty_cache()
    pb = pass_bytes(n)
    passes = pass_table(timing, pb)
    roof = roofline_of(passes, pb, MEASURED_TRAFFIC_512, n, tuning)
    roof["measured"] = (f"HIP events at kernel start/end, one lane, {reps} forward transforms and {reps} "
                        f"evaluations at alpha = {alpha:g}")
    return {"grid": n, "padded": 2 * n, "tile_shifts": tuning, "roofline": roof, "passes": passes}


def run_mode(ctx, torch, Fs, deltas, V0, opts, steps, warmup, timing=False):
    zs = [torch.empty_like(F) for F in Fs]
    cs = [torch.empty_like(F) for F in Fs]
    reps = None
    for _ in range(warmup):
        reps = ctx.solve_batch(Fs, deltas, zs, opts=opts, V0=V0, c0=1.0, c_list=cs)
    torch.cuda.synchronize()
    if timing:
        ctx.set_timing(True)
        for p in range(6):
            ctx.get_timing(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals, flags = [], []
    for _ in range(steps):
        reps = ctx.solve_batch(Fs, deltas, zs, opts=opts, V0=V0, c0=1.0, c_list=cs)
        evals += [r["n_evals"] for r in reps]
        flags += [r["flags"] for r in reps]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing_out = None
    if timing:
        timing_out = {PASS_NAMES[p]: ctx.get_timing(p) for p in range(6)}
        ctx.set_timing(False)
    el = t1 - t0
    n = len(Fs) * steps
    reached = sum(1 for f in flags if (f & 3) == 0)
    return dict(solves_per_s=n / el, ms_per_step=el / steps * 1e3, mean_evals=sum(evals) / len(evals),
                reached_delta_frac=reached / len(flags),
                noroot_low=sum(1 for f in flags if f & 2) / len(flags),
                fallback_frac=sum(1 for f in flags if f & 16) / len(flags)), timing_out, zs, reps


def fp64_section(torch, fr3d, Fs, deltas, net, learned_opts, bisect_opts, lanes, steps=2, warmup=1):
    """The same batch solved in FP64 throughout (the paper's arithmetic,
    Sec. 6): transforms, filter, norms and search in double, the learned
    search with the headline's network and options, and bisection; forward
    transform + search + recovery of c per solve, as the headline step."""
    n = Fs[0].shape[0]
    c = fr3d.Context(0)
    c.load_kernel(n, n, n, precision=64)
    c.apply_tuning(batched=True)
    c.set_lanes(lanes)
    c.predictor_set(*net)
    V = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    c.source_potential(V, 1.0)
    F64 = [F.double() for F in Fs]
    out = {}
    zs64 = reps64 = None
    for name, o in (("learned", learned_opts), ("bisection", bisect_opts)):
        r, _, zs, reps = run_mode(c, torch, F64, deltas, V, o, steps, warmup)
        out[name] = r
        if name == "learned":
            zs64, reps64 = zs, reps
    out["speedup_learned_vs_bisection_tol_1e-3"] = out["learned"]["solves_per_s"] / out["bisection"]["solves_per_s"]
    c.close()
    return out, zs64, reps64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--lanes", type=int, default=8)
    ap.add_argument("--predictor", default=os.path.join(ROOT, "paper_1703_01216_amd", "data", "predictor.bin"))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16, help="oracle processes of the CPU baseline")
    ap.add_argument("--graphs", type=int, default=0, help="1: replay each lane's evaluation as a HIP graph")
    ap.add_argument("--modes", default="learned,bisection,learned_ratio,learned_net,learned_w,bisection_w,kary16")
    ap.add_argument("--calibrate", type=int, default=96,
                    help="instances (not timed) on which the network is fine-tuned for this geometry; 0: none")
    ap.add_argument("--fp64", type=int, default=1, help="solve the batch in FP64 too")
    ap.add_argument("--n512", type=int, default=1, help="single-lane pass timing at 256^3 -> 512^3")
    ap.add_argument("--w3", type=int, default=64, help="instances of the uneven-size batched workload (0: skip)")
    ap.add_argument("--layered", type=int, default=1, help="time the per-frequency z-system form at the paper's size")
    ap.add_argument("--exact", type=int, default=1, help="time the exact-operator CG solve on one instance")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the single-lane kernel-timing sections (for profiler runs)")
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
        print(json.dumps({"copy": copy, "copy_sweep": copy_sweep(torch)}))
        return
    n = args.n
    ctx = fr3d.Context(0)
    ctx.load_kernel(n, n, n, precision=32)
    tuning = ctx.apply_tuning(batched=True)  # the headline and its kernels' single-lane timing
    ctx.set_lanes(args.lanes)
    ctx.set_graphs(bool(args.graphs))
    modes = args.modes.split(",")
    net_base = net_tuned = None
    if any(m.startswith("learned") for m in modes):
        if not os.path.exists(args.predictor):
            print(f"[bench] no predictor at {args.predictor}; skipping the learned searches", file=sys.stderr)
            modes = [m for m in modes if not m.startswith("learned")]
        else:
            ctx.predictor_load(args.predictor)
            net_base = ctx.predictor_get()
    Fs, deltas, V0 = make_instances(ctx, torch, n, args.batch)
    print(f"[bench] {len(Fs)} instances of {n}^3 ready", file=sys.stderr, flush=True)
    tight = dict(tol=1e-3, accept_lo=1 - 1e-3, accept_hi=1 + 1e-3)
    wide = dict(tol=0.1, accept_lo=0.9, accept_hi=1.1)
    # the network alone: the secant refinement assumes the median slope of
    # ln r at the root over training instances (recorded beside the checkpoint)
    meta = os.path.splitext(args.predictor)[0] + ".json"
    train_slope = json.load(open(meta))["root_slope"]["median"] if os.path.exists(meta) else 0.05
    # the headline learned search: the network fine-tuned on the GPU for this
    # geometry on instances of the same recipe that are not timed (indices
    # from CAL_FIRST), its median root slope and held-out seed spread
    sk, cal = {"seed_slope": train_slope}, None
    if net_base is not None and args.calibrate:
        from paper_1703_01216_amd import calibrate
        Fc, dc, _ = make_instances(ctx, torch, n, args.calibrate, first=CAL_FIRST)
        cal = calibrate.fine_tune(ctx, Fc, dc)
        cal["first_index"] = CAL_FIRST
        del Fc
        net_tuned = ctx.predictor_get()
        sk = {k: cal[k] for k in ("seed_slope", "seed_snap_lo", "seed_slope_ratio")}
        print(f"[bench] fine-tuning for the geometry: {cal}", file=sys.stderr, flush=True)
    # the headline: the fine-tuned seed, the first secant step with the fixed
    # median slope.  With the level features the seed is accepted at once for
    # most instances, and the whole-box slope (learned_ratio) would cost every
    # seed evaluation its reduction for the few that take a step.
    fixed = {**sk, "seed_slope_ratio": 0.0}
    mode_opts = {"learned": fr3d.default_opts(use_predictor=1, **fixed, **tight),
                 "learned_net": fr3d.default_opts(use_predictor=1, seed_slope=train_slope, **tight),
                 "learned_ratio": fr3d.default_opts(use_predictor=1, **sk, **tight),
                 "bisection": fr3d.default_opts(**tight),
                 "learned_w": fr3d.default_opts(use_predictor=1, **fixed, **wide),
                 "bisection_w": fr3d.default_opts(**wide)}
    for m in modes:
        if m.startswith("kary"):  # kary<K>: the K-candidate search
            mode_opts[m] = fr3d.default_opts(candidates=int(m[4:]), **tight)
    results, kept = {}, {}
    head = modes[0]
    if not args.roofline_only:
        for m in modes:
            if m.startswith("learned"):
                # learned_net: the shipped network alone (no fine-tuning)
                net = net_base if (m == "learned_net" or net_tuned is None) else net_tuned
                ctx.predictor_set(*net)
            r, _, zs, reps = run_mode(ctx, torch, Fs, deltas, V0, mode_opts[m], args.steps, args.warmup)
            results[m] = r
            if m == head:
                kept = {"zs": zs, "reps": reps}
            else:
                del zs
            print(f"[bench] {m}: {r}", file=sys.stderr, flush=True)
    timing, kt_el = kernel_timing(ctx, torch, Fs, deltas, mode_opts["bisection"], args.lanes)
    print(f"[bench] kernel timing section: {kt_el * 1e3:.1f} ms", file=sys.stderr, flush=True)
    pb = pass_bytes(n)
    passes = pass_table(timing, pb)
    roofline = roofline_of(passes, pb, MEASURED_TRAFFIC, n, tuning)
    roofline["measured"] = "HIP events at kernel start/end, one lane, bisection to 1e-3 over the batch"
    s512 = None
    if args.n512:
        s512 = section_512(torch, fr3d)
        print(f"[bench] 512^3 passes: {s512}", file=sys.stderr, flush=True)
    if args.roofline_only:
        print(json.dumps({"roofline": roofline, "passes": passes, "roofline_512": s512}))
        return
    H = results[head]
    out = {
        "metric": METRIC, "value": H["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": H["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n}^3 grids padded to {2 * n}^3, batch of {len(Fs)} instances (5-10 inclusions, "
                               f"delta 1/3/5%), forward transform + {head} alpha search to |r/delta - 1| <= 1e-3 "
                               f"+ recovery of c per solve, {args.lanes} lanes",
                   "grid": n, "padded": 2 * n, "batch": len(Fs), "lanes": args.lanes, "search": head,
                   "graphs": bool(args.graphs),
                   "tile_shifts": tuning,
                   "modes": results, "fine_tuning": cal, "train_root_slope": train_slope},
        "roofline": roofline,
        "roofline_512": s512["roofline"] if s512 else None,
        "passes": passes,
        "passes_512": s512["passes"] if s512 else None,
        "copy": copy,
    }
    per_solve = sum(pb[k] for k in ("fwd_x", "fwd_y", "fwd_z")) + 2 * n ** 3 * 4 * 2
    per_eval = sum(pb[k] for k in ("inv_z", "inv_y", "inv_x"))
    out["config"]["aggregate_GB_s"] = H["solves_per_s"] * (per_solve + H["mean_evals"] * per_eval) / 1e9
    if "learned" in results and "bisection" in results:
        out["config"]["speedup_learned_vs_bisection_tol_1e-3"] = (
            results["learned"]["solves_per_s"] / results["bisection"]["solves_per_s"])
    if "learned_net" in results and "bisection" in results:
        out["config"]["speedup_network_alone_vs_bisection_tol_1e-3"] = (
            results["learned_net"]["solves_per_s"] / results["bisection"]["solves_per_s"])
    if "learned_w" in results and "bisection_w" in results:
        out["config"]["speedup_learned_vs_bisection_tol_0.1"] = (
            results["learned_w"]["solves_per_s"] / results["bisection_w"]["solves_per_s"])
    if cal is not None and "learned" in results:
        # the fine-tuning is paid once per geometry: the learned solves it takes to repay
        out["config"]["fine_tuning_in_learned_solves"] = cal["seconds"] * results["learned"]["solves_per_s"]
    z64 = rep64 = None
    if args.fp64 and "learned" in results and "bisection" in results:
        net = net_tuned or net_base
        out["config"]["fp64"], z64, rep64 = fp64_section(torch, fr3d, Fs, deltas, net, mode_opts["learned"],
                                                         mode_opts["bisection"], args.lanes)
        print(f"[bench] fp64: {out['config']['fp64']}", file=sys.stderr, flush=True)
    if args.exact:
        out["config"]["exact_cg"] = exact_section(torch, fr3d, Fs, n)
        print(f"[bench] exact: {out['config']['exact_cg']}", file=sys.stderr, flush=True)
    # host copies for the oracle legs (first instances of the timed batch)
    n_cpu = min(len(Fs), max(4, args.cpu_workers))
    Fh = [F.double().cpu().numpy() for F in Fs[:n_cpu]]
    checks = []
    if kept:
        for i in range(min(4, len(Fs))):
            r = kept["reps"][i]
            checks.append({"kind": "check", "precision": 32, "index": i, "F": Fh[i], "delta": deltas[i],
                           "alpha": r["alpha"], "zeta": kept["zs"][i].double().cpu().numpy(),
                           "residual": r["residual"]})
            if z64 is not None:
                checks.append({"kind": "check", "precision": 64, "index": i, "F": Fh[i], "delta": deltas[i],
                               "alpha": rep64[i]["alpha"], "zeta": z64[i].cpu().numpy(),
                               "residual": rep64[i]["residual"]})
    kept = None
    del z64
    if args.w3 > 0:
        del Fs, V0
        torch.cuda.empty_cache()
        out["config"]["workload3"] = workload3_section(torch, fr3d, n_inst=args.w3)
        print(f"[bench] workload3: {out['config']['workload3']}", file=sys.stderr, flush=True)
    if args.layered:
        out["config"]["layered"] = layered_section(torch, fr3d)
        print(f"[bench] layered: {out['config']['layered']}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        net = net_tuned or net_base
        net_arg = (net[0].astype("float64"), net[1].astype("float64"), fixed) if net is not None else None
        cb = cpu_baseline(Fh, deltas[:n_cpu], net_arg, checks, workers=args.cpu_workers)
        res = cb.pop("precision_checks")
        out["precision"] = [dict(precision=c["precision"], index=c["index"], alpha=c["alpha"], **r)
                            for c, r in zip(checks, res)]
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
