"""What the trained network gains over the method without it (GPU, through
the C-ABI).  Held-out instances of the predictor's training recipe
(workload 5 at n = 64, every q; indices from 500000, disjoint from the
training instances 0 ... 19999) are solved by plain bisection and by the
learned search.  The learned search uses the shipped network and secant
steps with the training instances' median slope, without calibration.  Both
solve to |r/delta - 1| <= 1e-3:

* both reach the target on the same instances, and every answer is within
  the tolerance;
* the learned search takes at most half of bisection's evaluations on
  average;
* on one sampled instance, the FP64 oracle's residual at the learned alpha
  is within the tolerance (plus the FP32 path's rounding).
"""
import json
import os

import numpy as np
import pytest

from oracle import tikhonov
from oracle.geometry import sample_kernel

from gpu_helpers import geom

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 64
COUNT = 32
FIRST = 500000


@pytest.fixture(scope="module")
def fr3d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_01216_amd import fr3d as m
    return m


def held_out_recipes():
    from paper_1703_01216_amd import inputs
    out, i = [], FIRST
    while len(out) < COUNT:
        r = inputs.workload_params(5, i)
        if r["shape"] == (N, N, N):
            out.append(r)
        i += 1
    return out


def test_learned_search_gains_over_bisection(fr3d):
    from paper_1703_01216_amd import train
    here = os.path.dirname(fr3d.__file__)
    ckpt = os.path.join(here, "data", "predictor.bin")
    slope = json.load(open(os.path.join(here, "data", "predictor.json")))["root_slope"]["median"]
    tight = dict(tol=1e-3, accept_lo=1 - 1e-3, accept_hi=1 + 1e-3)
    by_q = {}
    for r in held_out_recipes():
        by_q.setdefault(r["q"], []).append(r)
    ev_b, ev_l, sample = [], [], None
    for q, recipes in sorted(by_q.items()):
        c = fr3d.Context()
        c.load_kernel(N, N, N, q=q, precision=32)
        c.predictor_load(ckpt)
        V0 = torch.empty((N, N, N), dtype=torch.float32, device="cuda")
        c.source_potential(V0)
        Fs, deltas = train.synthesize(c, torch, recipes, V0)
        for F, d in zip(Fs, deltas):
            z_b, z_l = torch.empty_like(F), torch.empty_like(F)
            c.set_data(F, d)
            rb = c.solve_discrepancy(z_b, **tight)
            c.set_data(F, d)
            rl = c.solve_discrepancy(z_l, use_predictor=1, seed_slope=slope, **tight)
            print("q", q, "delta", d, "bisection", rb["n_evals"], rb["flags"], "learned", rl["n_evals"], rl["flags"],
                  flush=True)
            assert (rb["flags"] & 3) == (rl["flags"] & 3)
            if rb["flags"] & 3 == 0:
                assert abs(rb["residual"] / d - 1) <= 1e-3 and abs(rl["residual"] / d - 1) <= 1e-3
                if sample is None:
                    sample = (q, F.cpu().numpy().astype(np.float64), d, rl["alpha"])
            ev_b.append(rb["n_evals"])
            ev_l.append(rl["n_evals"])
        c.close()
    mb, ml = float(np.mean(ev_b)), float(np.mean(ev_l))
    print(f"mean evaluations: bisection {mb:.2f}, learned {ml:.2f} ({mb / ml:.2f}x fewer)", flush=True)
    assert ml <= 0.5 * mb
    # the oracle's residual at the learned alpha of one instance
    q, Fh, d, alpha = sample
    g = geom(N, N, N, q=q)
    ref = tikhonov.solve_spectral(g, np.fft.fftn(sample_kernel(g)), Fh, alpha)
    assert abs(ref["r_norm"] / d - 1) <= 1e-3 + 2e-5
