"""Training of the alpha predictor on instances the method generates, on the GPU.

    python -m paper_1703_01216_amd.train --instances 20000 --out predictor.bin

Each instance of the training workload (inputs.workload_params(5, i): a
cubic grid of 64, 96 or 128 cells, source parameter q in {0..3} with its own
kernel, noise level U[0.5%, 5%]) is synthesised through the library's own
forward operator: zeta = xi V0 on R, F = A zeta on Y, plus seeded noise scaled
to delta.  Its label is log10 alpha* of the discrepancy search (bisection to
|r/delta - 1| <= 1e-6, i.e. the root) and its features are the 65 spectral features of F;
both come from the batch solver.  The network is then trained with the
library's BF16-MFMA kernels (Adam, mean squared error on standardised
log10 alpha) and saved as a checkpoint.  All of this runs through the C-ABI;
torch supplies device memory, the seeded noise draws and the field of the
inclusions.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1703_01216_amd import fr3d, inputs  # noqa: E402

DEFAULT_CKPT = os.path.join(HERE, "data", "predictor.bin")


def he_init(seed):
    import numpy as np
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for shape in ((128, 65), (128,), (128, 128), (128,), (128,), (1,)):
        if len(shape) == 1:
            parts.append(np.zeros(shape))
        else:
            lim = math.sqrt(6.0 / shape[1])
            parts.append(g.uniform(-lim, lim, size=shape))
    w3_lim = math.sqrt(6.0 / 128)
    parts[4] = g.uniform(-w3_lim, w3_lim, size=(128,))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def synthesize(ctx, torch, recipes, V0):
    """F and delta of each recipe through the context's forward operator."""
    Fs, deltas = [], []
    for r in recipes:
        xi = inputs.xi_torch(r["shape"], r["inclusions"])
        F = torch.empty_like(xi)
        ctx.apply_operator(xi * V0, F)
        e = inputs.noise_torch(r["shape"], r["seed"])
        deltas.append(ctx.add_noise(F, e, r["delta_rel"]))
        Fs.append(F)
    return Fs, deltas


def label_groups(indices, lanes=8, chunk=64, log=print, tol=1e-6, max_steps=60):
    """Features, labels and reports of workload-5 instances, grouped by (n, q)."""
    import numpy as np
    import torch

    recipes = {i: inputs.workload_params(5, i) for i in indices}
    groups = {}
    for i, r in recipes.items():
        groups.setdefault((r["shape"][0], r["q"]), []).append(i)
    X = np.zeros((len(indices), 65), np.float32)
    t = np.zeros(len(indices), np.float64)
    meta = {}
    pos = {i: k for k, i in enumerate(indices)}
    t0 = time.time()
    done = 0
    for (n, q), idx in sorted(groups.items()):
        ctx = fr3d.Context()
        ctx.load_kernel(n, n, n, q=q, precision=32)
        ctx.set_lanes(lanes)
        V0 = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        ctx.source_potential(V0)
        for s in range(0, len(idx), chunk):
            part = idx[s:s + chunk]
            Fs, deltas = synthesize(ctx, torch, [recipes[i] for i in part], V0)
            zs = [torch.empty_like(F) for F in Fs]
            feat = torch.empty((len(part), 65), dtype=torch.float32, device="cuda")
            reps = ctx.solve_batch(Fs, deltas, zs, feat=feat, tol=tol, max_steps=max_steps)
            fh = feat.cpu().numpy()
            for k, i in enumerate(part):
                X[pos[i]] = fh[k]
                t[pos[i]] = math.log10(reps[k]["alpha"])
                meta[i] = dict(n=n, q=q, delta_rel=recipes[i]["delta_rel"], flags=reps[k]["flags"],
                               n_evals=reps[k]["n_evals"])
            done += len(part)
            del Fs, zs
        log(f"[label] n={n} q={q}: {len(idx)} instances, total {done}/{len(indices)} in {time.time() - t0:.1f}s")
        ctx.close()
        del V0
        torch.cuda.empty_cache()
    return X, t, meta


def fit(X_tr, t_tr, X_va, t_va, epochs=150, batch=256, lr=1e-3, seed=1, log=print):
    """Train the network on the GPU; returns (context holding it, history)."""
    import numpy as np
    import torch

    mu = X_tr.mean(axis=0)
    sd = X_tr.std(axis=0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    tmu, tsd = float(t_tr.mean()), float(max(t_tr.std(), 1e-3))
    norm = np.concatenate([mu, sd, [tmu, tsd]]).astype(np.float32)
    ctx = fr3d.Context()
    ctx.predictor_set(he_init(seed), norm)
    Xd = torch.tensor(X_tr, device="cuda")
    td = torch.tensor(t_tr.astype(np.float32), device="cuda")
    Xv = torch.tensor(X_va, device="cuda")
    yv = torch.empty(len(X_va), dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    hist = []
    nb = max(1, len(X_tr) // batch)
    for ep in range(epochs):
        perm = torch.randperm(len(X_tr), generator=g, device="cuda")
        acc = 0.0
        step_lr = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)))  # cosine decay
        for b in range(nb):
            sel = perm[b * batch:(b + 1) * batch]
            ctx.predictor_train_step(Xd[sel].contiguous(), td[sel].contiguous(), step_lr, loss, None)
            acc += float(loss.item()) if b == nb - 1 else 0.0
        ctx.predictor_forward(Xv, yv)
        mae = float(np.abs(yv.cpu().numpy() - t_va).mean())
        hist.append(dict(epoch=ep, last_batch_loss=acc, val_mae_decades=mae))
        if ep % 10 == 0 or ep == epochs - 1:
            log(f"[fit] epoch {ep}: loss {acc:.4f} val MAE {mae:.3f} decades")
    return ctx, hist


def root_slopes(indices, ckpt, h=0.05, log=print):
    """d ln r / d log10 alpha at the discrepancy root of workload-5 instances
    (central difference over +-h decades around the root found by the batch
    solver to 1e-6), with the predictor's clipped seed t0 and the noise
    feature x_64 of each; instances without a root inside the range are
    skipped.  Their median is the default slope of the seeded search's secant
    refinement (calibrate.py fits one geometry more closely)."""
    import numpy as np
    import torch

    recipes = {i: inputs.workload_params(5, i) for i in indices}
    groups = {}
    for i, r in recipes.items():
        groups.setdefault((r["shape"][0], r["q"]), []).append(i)
    rows = []
    for (n, q), idx in sorted(groups.items()):
        ctx = fr3d.Context()
        ctx.load_kernel(n, n, n, q=q, precision=32)
        ctx.predictor_load(ckpt)
        V0 = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        ctx.source_potential(V0)
        Fs, deltas = synthesize(ctx, torch, [recipes[i] for i in idx], V0)
        z = torch.empty_like(Fs[0])
        y = torch.empty(1, dtype=torch.float32, device="cuda")
        for F, d in zip(Fs, deltas):
            ctx.set_data(F, d)
            feat, _ = ctx.get_features()
            ctx.predictor_forward(feat.view(1, 65).contiguous(), y)
            t0 = min(max(float(y[0]), -8.0), 0.0)
            x64 = float(feat[64])
            rep = ctx.solve_discrepancy(z, tol=1e-6, max_steps=60)
            if rep["flags"] != 0:
                continue
            t = math.log10(rep["alpha"])
            rp = ctx.solve_alpha(10.0 ** (t + h), z)["residual"]
            rm = ctx.solve_alpha(10.0 ** (t - h), z)["residual"]
            rows.append((t0, x64, (math.log(rp) - math.log(rm)) / (2 * h)))
        log(f"[slope] n={n} q={q}: {len(idx)} instances")
        ctx.close()
        del V0, Fs
        torch.cuda.empty_cache()
    return np.array(rows)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--lanes", type=int, default=8)
    ap.add_argument("--out", default=DEFAULT_CKPT)
    ap.add_argument("--first-index", type=int, default=0)
    ap.add_argument("--label-tol", type=float, default=1e-6)
    ap.add_argument("--predictor", default=DEFAULT_CKPT, help="checkpoint whose seeds the slope model uses")
    ap.add_argument("--root-slope", type=int, default=0,
                    help="only measure the residual slope at the root on this many training instances and "
                         "record its median in the checkpoint's JSON summary")
    args = ap.parse_args(argv)
    import numpy as np
    import torch

    torch.cuda.set_device(0)
    log = lambda m: print(m, flush=True)  # noqa: E731
    meta_path = os.path.splitext(args.out)[0] + ".json"
    if args.root_slope:
        rows = root_slopes(list(range(args.first_index, args.first_index + args.root_slope)), args.predictor,
                           log=log)
        sl = rows[:, 2]
        summary = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
        summary["root_slope"] = dict(median=float(np.median(sl)), q25=float(np.percentile(sl, 25)),
                                     q75=float(np.percentile(sl, 75)), instances=int(sl.size),
                                     first_index=args.first_index)
        with open(meta_path, "w") as fh:
            json.dump(summary, fh, indent=1)
        log(json.dumps(summary["root_slope"]))
        return
    n = args.instances
    idx = list(range(args.first_index, args.first_index + n))
    X, t, meta = label_groups(idx, lanes=args.lanes, log=log, tol=args.label_tol)
    n_va = max(1, n // 20)
    n_te = max(1, n // 20)
    n_tr = n - n_va - n_te
    ctx, hist = fit(X[:n_tr], t[:n_tr], X[n_tr:n_tr + n_va], t[n_tr:n_tr + n_va], epochs=args.epochs, log=log)
    y = torch.empty(n_te, dtype=torch.float32, device="cuda")
    ctx.predictor_forward(torch.tensor(X[n - n_te:], device="cuda"), y)
    err = y.cpu().numpy() - t[n - n_te:]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    ctx.predictor_save(args.out)
    flags = np.array([meta[i]["flags"] for i in idx])
    summary = dict(instances=n, split=[n_tr, n_va, n_te], first_index=args.first_index, epochs=args.epochs,
                   label_tol=args.label_tol,
                   test_mae_decades=float(np.abs(err).mean()),
                   test_within_0_25_decades=float((np.abs(err) <= 0.25).mean()),
                   test_within_0_05_decades=float((np.abs(err) <= 0.05).mean()),
                   label_flags={str(k): int((flags == k).sum()) for k in sorted(set(flags.tolist()))},
                   label_mean_evals=float(np.mean([meta[i]["n_evals"] for i in idx])),
                   last=hist[-1])
    with open(meta_path, "w") as fh:
        json.dump(summary, fh, indent=1)
    log(json.dumps(summary))


if __name__ == "__main__":
    main()
