"""Seeded synthetic weight tensors for the benchmark and test workloads.

Holds no arithmetic of the method: only random draws (NumPy PCG64 via
``numpy.random.default_rng``) and the layer shapes.  Both the oracle-side
tests and the GPU path take their inputs from here.

Every tensor is drawn in C order ``[c_out, c_in, kh, kw]`` as
``standard_normal * std`` in float64 and then cast to the workload's dtype.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Layer:
    c_out: int
    c_in: int
    kh: int
    kw: int
    n: int
    m: int

    @property
    def r(self) -> int:
        return min(self.c_out, self.c_in)

    @property
    def num_sigma(self) -> int:
        return self.n * self.m * self.r


def gaussian(rng, shape, std, dtype):
    return (rng.standard_normal(shape) * std).astype(dtype)


def single_layer_16(seed: int = 0):
    """16 -> 16 channels, 3x3 kernel, 32x32 periodic grid, float64 weights
    N(0, 1/(9*16))."""
    L = Layer(16, 16, 3, 3, 32, 32)
    rng = np.random.default_rng(seed)
    W = gaussian(rng, (16, 16, 3, 3), np.sqrt(1.0 / (9 * 16)), np.float64)
    return L, W


def brute_force_small(seed: int = 1):
    """4 -> 4 channels, 3x3, 8x8 grid (dense operator 256 x 256), float64."""
    L = Layer(4, 4, 3, 3, 8, 8)
    rng = np.random.default_rng(seed)
    W = gaussian(rng, (4, 4, 3, 3), np.sqrt(1.0 / (9 * 4)), np.float64)
    return L, W


def single_layer_64(seed: int = 2):
    """64 -> 64 channels, 3x3, 64x64 grid, float32 weights N(0, 1/(9*64))."""
    L = Layer(64, 64, 3, 3, 64, 64)
    rng = np.random.default_rng(seed)
    W = gaussian(rng, (64, 64, 3, 3), np.sqrt(1.0 / (9 * 64)), np.float32)
    return L, W


def rectangular_256_512(seed: int = 3):
    """256 -> 512 channels, 3x3, 32x32 grid, float32 weights N(0, 1/(9*256))."""
    L = Layer(512, 256, 3, 3, 32, 32)
    rng = np.random.default_rng(seed)
    W = gaussian(rng, (512, 256, 3, 3), np.sqrt(1.0 / (9 * 256)), np.float32)
    return L, W


def _round_significand(x, bits):
    """Round to ``bits`` significant bits (so products of two such numbers are
    exact in float32's 24-bit significand when 2*bits <= 24)."""
    mant, expo = np.frexp(x)
    return np.ldexp(np.round(np.ldexp(mant, bits)), expo - bits)


def rank_one_taps(c_out: int = 512, c_in: int = 256, k: int = 3, n: int = 32, seed: int = 31):
    """Every tap is exactly rank one in float32:
    ``W[:, :, a, b] = a_y b_y^T`` with ``a_y ~ N(0, 1/(k*k*c_in))`` and
    ``b_y ~ N(0, 1)``, both rounded to 8 significant bits so that every
    product is exact in float32."""
    L = Layer(c_out, c_in, k, k, n, n)
    rng = np.random.default_rng(seed)
    a = _round_significand(rng.standard_normal((k, k, c_out)) / np.sqrt(k * k * c_in), 8)
    b = _round_significand(rng.standard_normal((k, k, c_in)), 8)
    W = np.einsum("abo,abi->oiab", a, b)
    W32 = np.ascontiguousarray(W, dtype=np.float32)
    assert np.array_equal(W32.astype(np.float64), W)
    return L, W32


RESNET18_CIFAR_SHAPES = (
    # (c_in, c_out, n)
    (3, 64, 32),
    (64, 64, 32), (64, 64, 32), (64, 64, 32), (64, 64, 32),
    (64, 128, 16), (128, 128, 16), (128, 128, 16),
    (128, 256, 8), (256, 256, 8),
    (256, 512, 4), (512, 512, 4),
)


def resnet18_stack(seed: int = 4, shapes=RESNET18_CIFAR_SHAPES):
    """Twelve stride-1 periodic 3x3 layers with the channel counts and grid
    sizes of ResNet-18 on 32x32 inputs; float32 He-normal weights
    ``std = sqrt(2 / (c_in * 9))``, drawn in layer order from one generator."""
    rng = np.random.default_rng(seed)
    layers, weights = [], []
    for c_in, c_out, n in shapes:
        layers.append(Layer(c_out, c_in, 3, 3, n, n))
        weights.append(gaussian(rng, (c_out, c_in, 3, 3), np.sqrt(2.0 / (c_in * 9)), np.float32))
    return layers, weights


def large_grid_7x7(seed: int = 5, n: int = 224, scaled_taps: int = 5, scale: float = 1e3):
    """64 -> 64 channels, 7x7 kernel, n x n grid (224 by default), float32
    weights N(0, 1/(49*64)); ``scaled_taps`` of the 49 taps (a tap is the whole
    64x64 slice W[:, :, a, b]; 5 = round(10% of 49)) are multiplied by
    ``scale``.  Returns (layer, W, scaled tap indices a*7+b)."""
    L = Layer(64, 64, 7, 7, n, n)
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((64, 64, 7, 7)) * np.sqrt(1.0 / (49 * 64))
    taps = rng.choice(49, scaled_taps, replace=False)
    for t in taps:
        W[:, :, t // 7, t % 7] *= scale
    return L, W.astype(np.float32), np.sort(taps)


def paper_scale(n: int, seed: int = 6):
    """16 -> 16 channels, 3x3, n x n grid, float32 weights N(0, 1/(9*16)):
    the channel count and kernel of the runtime study (Sec. IV, Tables II
    and III), sigma only, n up to 16384."""
    L = Layer(16, 16, 3, 3, n, n)
    rng = np.random.default_rng(seed)
    W = gaussian(rng, (16, 16, 3, 3), np.sqrt(1.0 / (9 * 16)), np.float32)
    return L, W


def resnet18_downsampling(seed: int = 7):
    """The stride-2 layers where ResNet-18 on 32x32 inputs first halves its
    grid: the 3x3 convolution 64 -> 128 and the 1x1 shortcut 64 -> 128, both
    on the 32x32 input grid, float32 He-normal.  Returns a list of
    (name, layer, stride, W)."""
    rng = np.random.default_rng(seed)
    out = []
    for name, k in (("3x3", 3), ("1x1_shortcut", 1)):
        L = Layer(128, 64, k, k, 32, 32)
        out.append((name, L, 2, gaussian(rng, (128, 64, k, k), np.sqrt(2.0 / (64 * k * k)), np.float32)))
    return out


def graded_channels(c_out, c_in, kh, kw, n, m=None, scales=(1.0, 10 ** 2.5, 1e5), seed=0,
                    dtype=np.float32):
    """N(0, 1/(kh*kw*c_in)) layer whose input channel i is multiplied by
    ``scales[i % len(scales)]``: every symbol's columns (of the tall layer)
    are graded by those factors, singular values spread over their range."""
    m = n if m is None else m
    L = Layer(c_out, c_in, kh, kw, n, m)
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((c_out, c_in, kh, kw)) * np.sqrt(1.0 / (kh * kw * c_in))
    W *= np.asarray([scales[i % len(scales)] for i in range(c_in)])[None, :, None, None]
    return L, W.astype(dtype)


def random_layer(c_out, c_in, kh, kw, n, m=None, seed=0, dtype=np.float32):
    """Generic N(0, 1/(kh*kw*c_in)) layer for parity tests."""
    m = n if m is None else m
    L = Layer(c_out, c_in, kh, kw, n, m)
    rng = np.random.default_rng(seed)
    W = gaussian(rng, (c_out, c_in, kh, kw), np.sqrt(1.0 / (kh * kw * c_in)), dtype)
    return L, W
