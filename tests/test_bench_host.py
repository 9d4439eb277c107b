"""Host-side checks of bench.py (no GPU): the one-GPU guard and the
algorithmic bytes per pass launch, from the buffer sizes of the layout
(n^3 real on R/Y, half spectrum Kx = n + 1 planes, the octant read at the
path's precision)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("n,esz", [(16, 4), (128, 4), (16, 8)])
def test_pass_bytes_from_buffer_sizes(n, esz):
    P, kx = 2 * n, n + 1
    real, cpx = esz, 2 * esz              # real, complex of the path's precision
    F = n ** 3 * real                     # F on Y, zeta on R
    A = kx * n * n * cpx                  # x done
    B = kx * n * P * cpx                  # y done
    S = kx * P * P * cpx                  # spectrum
    O = kx * (n + 1) * (n + 1) * cpx      # octant of k^ as the filter reads it
    Lv = kx * (n + 1) * P                 # byte table of kernel-spectrum levels (features), rows over all kz
    W1 = kx * n * P * 2 * cpx             # (u^, r^) pairs, z undone
    W2 = kx * n * n * 2 * cpx             # (u^, r^) pairs, y undone
    want = {"fwd_x": F + A, "fwd_y": A + B, "fwd_z": B + S + Lv, "inv_z": S + O + W1, "inv_y": W1 + W2,
            "inv_x": W2 + F}
    assert bench.pass_bytes(n, esz) == want
    if n == 128:  # the figures quoted for the bench workload
        mb = {k: round(v / 1e6, 1) for k, v in want.items()}
        assert mb == {"fwd_x": 25.3, "fwd_y": 50.7, "fwd_z": 105.7, "inv_z": 152.4, "inv_y": 101.4, "inv_x": 42.2}
