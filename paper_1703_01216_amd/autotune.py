"""Autotuner of the pass kernels' tile sizes.

    python -m paper_1703_01216_amd.autotune --sizes 128,64,96,192,256 [--out data/tuning.json]

For each padded geometry and precision, every pass is timed (HIP events at
the kernel's own start and end) with each of its tile variants -- a 32 KiB
LDS tile of pencils, half of it, and for the row passes a quarter -- while
the other passes keep their default, and the fastest variant is kept (the
inverse z pass also has a joint variant: half the ky columns with u^ and r^
transformed together).  The
result is a JSON cache {"<Px>x<Py>x<Pz>/fp<precision>": {pass: shift}} that
fr3d.Context.apply_tuning() applies; results do not depend on the choice.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1703_01216_amd import fr3d  # noqa: E402

SHIFTS = {"fwd_x": (0, 1, 2), "fwd_y": (0, 1, 2), "fwd_z": (0, 1), "inv_z": (0, 1, 2), "inv_y": (0, 1, 2), "inv_x": (0, 1)}


def tune_geometry(n, precision=32, reps=20, log=print):
    import torch
    ctx = fr3d.Context()
    ctx.load_kernel(n, n, n, precision=precision)
    dt = torch.float64 if precision == 64 else torch.float32
    g = torch.Generator(device="cuda")
    g.manual_seed(n)
    F = torch.randn((n, n, n), generator=g, device="cuda", dtype=dt)
    zeta = torch.empty_like(F)
    ctx.set_data(F, float(F.norm()) * 0.02)
    best, table = {}, {}
    for name, shifts in SHIFTS.items():
        pid = fr3d.PASS_NAMES.index(name)
        times = {}
        for sh in shifts:
            ctx.set_tile(pid, sh)
            ctx.set_data(F, 1.0)
            ctx.solve_alpha(1e-6, zeta)
            ctx.set_timing(True)
            for p in range(6):
                ctx.get_timing(p)
            for _ in range(reps):
                if pid < 3:
                    ctx.set_data(F, 1.0)
                else:
                    ctx.solve_alpha(1e-6, zeta)
            torch.cuda.synchronize()
            ms, cnt = ctx.get_timing(pid)
            ctx.set_timing(False)
            times[sh] = ms / max(cnt, 1) * 1e3
        ctx.set_tile(pid, 0)
        best[name] = min(times, key=times.get)
        table[name] = {str(k): round(v, 2) for k, v in times.items()}
        log(f"[tune] {2 * n}^3 fp{precision} {name}: " + ", ".join(f"shift {k}: {v:.2f} us" for k, v in times.items()))
    ctx.close()
    return best, table


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="128")
    ap.add_argument("--precisions", default="32")
    ap.add_argument("--out", default=fr3d.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    cache = json.load(open(args.out)) if os.path.exists(args.out) else {}
    report = {}
    for prec in (int(p) for p in args.precisions.split(",")):
        for n in (int(s) for s in args.sizes.split(",")):
            best, table = tune_geometry(n, prec, args.reps, log=lambda m: print(m, flush=True))
            key = f"{2 * n}x{2 * n}x{2 * n}/fp{prec}"
            cache[key] = best
            report[key] = table
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    print(json.dumps({"tuning": cache, "times_us": report}))


if __name__ == "__main__":
    main()
