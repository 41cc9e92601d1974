"""CPU checks of the benchmark's contract and cost formulas (no GPU)."""
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_cost_by_hand():
    """3x3 array, near radius 1 (9 near displacements), 16 far ones of rank 2,
    n = 80 macro RWG, n_a = 40, complex64 store."""
    L, n, n_a, nr = 3, 80, 40, 1
    store = SimpleNamespace(Dx=L - 1, near_radius=nr, near_dtype=1, n=n, ranks=np.full(16, 2))
    byt, flops, mean_rank = bench.algorithmic(store, L, n_a)
    pairs_near = sum((L - abs(dx)) * (L - abs(dy)) for dx in (-1, 0, 1) for dy in (-1, 0, 1))
    pairs_far = L ** 4 - pairs_near
    assert flops == 8.0 * n_a ** 2 * pairs_near + 16.0 * 2 * n_a * pairs_far
    assert byt == 9 * n * n * 8 + 16 * 2 * n * 2 * 8 + 2 * L * L * n_a * 16 + L * L
    assert mean_rank == 2.0


def test_spectral_cost_grid():
    byt, flops, G = bench.spectral_cost(80, 127, 16)
    assert G == 256                      # smallest power of two >= 2 * 127 + 1
    assert byt == 80 * 80 * G * G * 8    # complex64 spectra read once
    assert flops > 8 * 80 * 80 * G * G * 16
