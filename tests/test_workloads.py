"""Host-side checks of the seeded workload recipes and of bench.py's
one-GPU contract (CPU only).

The recipes must reproduce the shapes, sizes and value distributions of the
configurations the benchmark and the parity tests are quoted on; these tests
pin the counts that follow from those shapes (symbols, singular values,
parameters) and the draw statistics, so that a changed shape or scale shows
up here rather than as a silently different benchmark.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402


def _std_ok(W, std, rel=0.05):
    return abs(float(np.std(W.astype(np.float64))) / std - 1.0) < rel


def test_recipes_are_deterministic_in_the_seed():
    for fn in (workloads.single_layer_16, workloads.single_layer_64, workloads.brute_force_small):
        a, b, c = fn(0)[1], fn(0)[1], fn(1)[1]
        assert np.array_equal(a, b)
        assert not np.array_equal(a, c)
    s1, s2 = workloads.resnet18_stack()[1], workloads.resnet18_stack()[1]
    assert all(np.array_equal(x, y) for x, y in zip(s1, s2))


def test_single_layer_recipes():
    L, W = workloads.single_layer_16()
    assert (L.c_out, L.c_in, L.kh, L.kw, L.n, L.m) == (16, 16, 3, 3, 32, 32)
    assert W.dtype == np.float64 and L.num_sigma == 16384 and L.n * L.m == 1024
    assert _std_ok(W, np.sqrt(1.0 / 144), rel=0.1)

    L, W = workloads.single_layer_64()
    assert (L.c_out, L.c_in, L.n, L.m) == (64, 64, 64, 64)
    assert W.dtype == np.float32 and L.n * L.m == 4096 and L.num_sigma == 262144
    assert _std_ok(W, np.sqrt(1.0 / 576))

    L, W = workloads.rectangular_256_512()
    assert (L.c_out, L.c_in, L.n) == (512, 256, 32)
    assert L.num_sigma == 262144 and _std_ok(W, np.sqrt(1.0 / (9 * 256)), rel=0.02)


def test_resnet18_stack_counts():
    layers, weights = workloads.resnet18_stack()
    assert len(layers) == 12
    assert sum(L.num_sigma for L in layers) == 384000
    assert sum(w.size for w in weights) == 4941504
    classes = {}
    for L in layers:
        key = (L.c_out, L.c_in)
        classes[key] = classes.get(key, 0) + L.n * L.m
    # (c_out, c_in) -> number of symbols of that shape
    assert classes == {(64, 3): 1024, (64, 64): 4096, (128, 64): 256, (128, 128): 512,
                       (256, 128): 64, (256, 256): 64, (512, 256): 16, (512, 512): 16}
    for L, w in zip(layers, weights):
        assert w.shape == (L.c_out, L.c_in, 3, 3) and w.dtype == np.float32
        if w.size >= 4096:
            assert _std_ok(w, np.sqrt(2.0 / (9 * L.c_in)))


def test_large_grid_scaled_taps():
    L, W, taps = workloads.large_grid_7x7(n=8)
    assert (L.c_out, L.c_in, L.kh, L.kw) == (64, 64, 7, 7)
    assert len(taps) == 5 and len(set(taps.tolist())) == 5
    norms = np.sqrt((W.astype(np.float64) ** 2).sum(axis=(0, 1))).reshape(-1)
    big = np.argsort(norms)[-5:]
    assert sorted(big.tolist()) == sorted(taps.tolist())
    # the scaled taps are 1e3 times larger in norm, to a few percent
    small = np.delete(norms, taps)
    assert 0.9e3 < norms[taps].mean() / small.mean() < 1.1e3


def test_rank_one_taps_are_exact_in_float32():
    L, W = workloads.rank_one_taps(c_out=16, c_in=8, n=8)
    for a in range(3):
        for b in range(3):
            assert np.linalg.matrix_rank(W[:, :, a, b].astype(np.float64)) == 1


def test_downsampling_layers():
    out = workloads.resnet18_downsampling()
    assert [name for name, *_ in out] == ["3x3", "1x1_shortcut"]
    for _, L, s, W in out:
        assert s == 2 and (L.c_out, L.c_in, L.n) == (128, 64, 32)
        assert W.shape == (128, 64, L.kh, L.kw)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    assert r.returncode == 2
    assert r.stdout.strip() == ""
    assert "single MI355X" in r.stderr
