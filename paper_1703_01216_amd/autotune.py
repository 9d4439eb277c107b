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

    python -m paper_1703_01216_amd.autotune --sizes 128 --batched 64

scores every candidate instead by the time per solve of a batch of B data
sets solved on `--lanes` lanes at once (solve_batch), each solve being what
the learned search does for most instances: the forward transform, the
features and the network's seed, one evaluation at the seed (accepted: the
acceptance window is made wide) and the recovery; one score for all six
passes.  Alone, a pass's fastest tile can be a half tile whose workgroups
share 128 B lines through an XCD's L2; with several lanes' kernels
competing for the caches, tiles that read and write whole lines can win.
The result goes to the key "<Px>x<Py>x<Pz>/fp<precision>/batch", which
Context.apply_tuning(batched=True) prefers.
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

PREDICTOR_PATH = os.path.join(HERE, "data", "predictor.bin")

SHIFTS = {"fwd_x": (0, 1, 2), "fwd_y": (0, 1, 2), "fwd_z": (0, 1), "inv_z": (0, 1, 2), "inv_y": (0, 1, 2), "inv_x": (0, 1)}
PLAN_LENGTHS = (192, 384, 512)  # lengths with radix plan variants (FP32)


def candidates(name, P, precision):
    """Codes (tile shift + 4 plan variant) a pass of transform length P has."""
    shifts = SHIFTS[name] if P >= 64 else (0,)
    plans = (0, 1, 2) if precision == 32 and P in PLAN_LENGTHS else (0,)
    return [sh + 4 * v for v in plans for sh in shifts]


def tune_geometry(n, precision=32, reps=20, sweeps=3, start=None, margin=0.01, log=print, batched=0, lanes=8):
    import time

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
    if batched:
        ctx.set_lanes(lanes)
        ctx.predictor_load(PREDICTOR_PATH)
        Fs = [torch.randn((n, n, n), generator=g, device="cuda", dtype=dt) for _ in range(batched)]
        deltas = [float(f.norm()) * 0.02 for f in Fs]
        zs = [torch.empty_like(f) for f in Fs]
        opts = fr3d.default_opts(use_predictor=1, accept_lo=1e-6, accept_hi=1e6)

    def score_batched():
        for k, v in choice.items():
            ctx.set_tile(fr3d.PASS_NAMES.index(k), v)
        ctx.solve_batch(Fs, deltas, zs, opts=opts)
        torch.cuda.synchronize()
        rounds = []
        for _ in range(3):
            t0 = time.perf_counter()
            for _ in range(max(1, reps // 10)):
                ctx.solve_batch(Fs, deltas, zs, opts=opts)
            torch.cuda.synchronize()
            rounds.append((time.perf_counter() - t0) / (max(1, reps // 10) * batched) * 1e6)
        rounds.sort()
        return rounds[1], {"us_per_solve": rounds[1]}

    def score(forward):
        if batched:
            return score_batched()
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
            log(f"[tune] {2 * n}^3 fp{precision}{' batched' if batched else ''} {name}: " + ", ".join(
                f"code {k}: {v:.2f} us" for k, v in times.items()) + f" -> {choice[name]}")
        if not changed:
            break
    if batched:
        total, per = score_batched()
        ctx.close()
        return dict(choice), {"candidates_us": table, "batched_us_per_solve": total}
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
    ap.add_argument("--batched", type=int, default=0,
                    help="B > 0: score by the time per solve of B data sets solved on --lanes lanes at once")
    ap.add_argument("--lanes", type=int, default=8)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    cache = json.load(open(args.out)) if os.path.exists(args.out) else {}
    report = {}
    for prec in (int(p) for p in args.precisions.split(",")):
        for n in (int(s) for s in args.sizes.split(",")):
            plain = f"{2 * n}x{2 * n}x{2 * n}/fp{prec}"
            key = plain + ("/batch" if args.batched else "")
            best, table = tune_geometry(n, prec, args.reps, args.sweeps, start=cache.get(key) or cache.get(plain),
                                        log=lambda m: print(m, flush=True), batched=args.batched,
                                        lanes=args.lanes)
            cache[key] = best
            report[key] = table
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    print(json.dumps({"tuning": cache, "times_us": report}))


if __name__ == "__main__":
    main()
