"""Autotuner of the pass kernels' tile sizes and radix plans.

    python -m paper_1703_01216_amd.autotune --sizes 128,64,96,192,256 [--out data/tuning.json]

For each padded geometry and precision, every pass kernel has tile variants
(a 32 KiB LDS tile of pencils, half of it, and for the row passes a
quarter; the inverse z pass also a joint variant: half the ky columns with
u^ and r^ transformed together) and, for the FP32 transforms of lengths 192,
384 and 512, three radix plans (orders of the stage radices).  The search is
a coordinate descent on whole transforms: a candidate of a forward pass is
scored by the summed time of the three forward passes, one of an inverse
pass by the summed time of the three inverse passes (HIP events at each
kernel's start and end), so a variant that is fast itself but leaves the next
pass slower loses; every candidate of every pass is tried with the others at
their current choice (a candidate replaces it only when faster by more than
`margin`, 1%, the timing noise), and the sweep over the passes repeats until
nothing changes (at most `sweeps` times).  The result is a JSON cache
{"<Px>x<Py>x<Pz>/fp<precision>": {pass: code}} with code = tile shift + 4 x
plan variant, which fr3d.Context.apply_tuning() applies; results do not
depend on the choice beyond rounding.
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
PLAN_LENGTHS = (192, 384, 512)  # lengths with radix plan variants (FP32)


def candidates(name, P, precision):
    """Codes (tile shift + 4 plan variant) a pass of transform length P has."""
    shifts = SHIFTS[name] if P >= 64 else (0,)
    plans = (0, 1, 2) if precision == 32 and P in PLAN_LENGTHS else (0,)
    return [sh + 4 * v for v in plans for sh in shifts]


def tune_geometry(n, precision=32, reps=20, sweeps=3, start=None, margin=0.01, log=print):
    import torch
    ctx = fr3d.Context()
    ctx.load_kernel(n, n, n, precision=precision)
    dt = torch.float64 if precision == 64 else torch.float32
    g = torch.Generator(device="cuda")
    g.manual_seed(n)
    F = torch.randn((n, n, n), generator=g, device="cuda", dtype=dt)
    zeta = torch.empty_like(F)
    ctx.set_data(F, float(F.norm()) * 0.02)
    choice = {k: 0 for k in SHIFTS}
    if start:
        choice.update({k: v for k, v in start.items() if v in candidates(k, 2 * n, precision)})

    def score(forward):
        for k, v in choice.items():
            ctx.set_tile(fr3d.PASS_NAMES.index(k), v)
        ctx.set_data(F, 1.0)
        ctx.solve_alpha(1e-6, zeta)
        ctx.set_timing(True)
        for p in range(6):
            ctx.get_timing(p)
        for _ in range(reps):
            if forward:
                ctx.set_data(F, 1.0)
            else:
                ctx.solve_alpha(1e-6, zeta)
        torch.cuda.synchronize()
        ids = (0, 1, 2) if forward else (3, 4, 5)
        per = {}
        for p in ids:
            ms, cnt = ctx.get_timing(p)
            per[fr3d.PASS_NAMES[p]] = ms / max(cnt, 1) * 1e3
        ctx.set_timing(False)
        return sum(per.values()), per

    table = {}
    for sweep in range(sweeps):
        changed = False
        for name in SHIFTS:
            forward = name.startswith("fwd")
            times = {}
            for code in candidates(name, 2 * n, precision):
                keep = choice[name]
                choice[name] = code
                times[code], _ = score(forward)
                choice[name] = keep
            best = min(times, key=times.get)
            if times[best] > (1.0 - margin) * times[choice[name]]:
                best = choice[name]  # within the timing noise of the current choice: keep it
            if best != choice[name]:
                changed = True
                choice[name] = best
            table[f"{name} (sweep {sweep})"] = {str(k): round(v, 2) for k, v in times.items()}
            log(f"[tune] {2 * n}^3 fp{precision} {name}: " + ", ".join(
                f"code {k}: {v:.2f} us" for k, v in times.items()) + f" -> {choice[name]}")
        if not changed:
            break
    total_f, per_f = score(True)
    total_i, per_i = score(False)
    ctx.close()
    return dict(choice), {"candidates_us": table, "forward_us": per_f, "evaluation_us": per_i}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="128")
    ap.add_argument("--precisions", default="32")
    ap.add_argument("--out", default=fr3d.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--sweeps", type=int, default=3)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    cache = json.load(open(args.out)) if os.path.exists(args.out) else {}
    report = {}
    for prec in (int(p) for p in args.precisions.split(",")):
        for n in (int(s) for s in args.sizes.split(",")):
            key = f"{2 * n}x{2 * n}x{2 * n}/fp{prec}"
            best, table = tune_geometry(n, prec, args.reps, args.sweeps, start=cache.get(key),
                                        log=lambda m: print(m, flush=True))
            cache[key] = best
            report[key] = table
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    print(json.dumps({"tuning": cache, "times_us": report}))


if __name__ == "__main__":
    main()
