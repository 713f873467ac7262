"""Host-side logic of the package that needs no GPU: storage accounting of the large run
and the PSNR reduction of the binding."""
import math

import numpy as np

from oracle import ndgi_oracle as O


def test_large_run_bits_per_texel_matches_oracle():
    from paper_2604_12625_amd.large import bits_per_texel
    for dims in ((4096, 4096, 1024, 1024, 48), (1024, 1024, 256, 256, 24), (64, 64, 16, 16, 8)):
        assert math.isclose(bits_per_texel(*dims), O.bits_per_texel_bc4_grid(*dims), rel_tol=1e-12)
    # 4096^2 x 48: 32 bits of BC4 per texel spread over 48 keys, plus 8 FP16 grid values per
    # 16 texels per key
    assert math.isclose(bits_per_texel(4096, 4096, 1024, 1024, 48),
                        32 / 48 + 8 + 1699 * 16 / (4096 * 4096 * 48), rel_tol=1e-12)


def test_bordered_training_samples_are_the_mirror_padded_tile():
    """Samples drawn with a border are positions of the mirror-padded tile folded back by
    mirror addressing: every texel inside the tile, and each texel drawn as often as it
    occurs in numpy's symmetric padding of the tile."""
    import torch
    from paper_2604_12625_amd import inputs as I
    W, H, T, b, n = 12, 8, 3, 4, 400_000
    s = I.train_samples_torch(n, W, H, T, seed=5, device="cpu", border=b).numpy()
    x, y, k = s & 0xFFF, (s >> 12) & 0xFFF, s >> 24
    assert x.min() >= 0 and x.max() < W and y.min() >= 0 and y.max() < H and k.max() < T
    wx = np.bincount(np.pad(np.arange(W), b, mode="symmetric"), minlength=W) / (W + 2 * b)
    wy = np.bincount(np.pad(np.arange(H), b, mode="symmetric"), minlength=H) / (H + 2 * b)
    fx, fy = np.bincount(x, minlength=W) / n, np.bincount(y, minlength=H) / n
    assert np.max(np.abs(fx - wx)) < 5e-3 and np.max(np.abs(fy - wy)) < 5e-3
    plain = I.train_samples_torch(1000, W, H, T, seed=5, device="cpu").numpy()
    assert (plain & 0xFFF).max() < W


def test_bench_measures_one_gpu_only():
    """bench.py --gpus N with N > 1 exits with a message (no multi-GPU path is built)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
