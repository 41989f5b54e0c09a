"""Host-only checks of the benchmark script: the one-GPU contract and the
network FLOP count it reports (counted here from the oracle's layer shapes)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import lesnet as N  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_network_flops_match_the_layer_shapes():
    """Forward: 2 multiply-adds per weight per output voxel of each layer
    (up layers: per coarse voxel and child); backward: the same for the
    weight gradients plus the input gradients of every layer but the
    first."""
    D, H, W = 8, 12, 16
    shp = N.shapes()
    vox = {"e1a": 1, "e1b": 1, "d1a": 1, "d1b": 1, "head": 1, "e2a": 8, "e2b": 8, "d2a": 8, "d2b": 8,
           "u1": 8, "b1": 64, "b2": 64, "u2": 64}
    m = D * H * W
    fwd = sum(2 * int(np.prod(s)) * (m // vox[k]) for k, s in shp.items())
    first = 2 * int(np.prod(shp["e1a"])) * m
    f, b = bench.net_flops(D, H, W)
    assert f == fwd
    assert b == 2 * fwd - first
