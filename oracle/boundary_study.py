"""Periodic (LFA) against zero-padded (Dirichlet) spectra of one layer.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper compares
the singular values LFA computes under periodic boundary conditions with
those of the same convolution under zero padding and finds them close, the
more so the larger the grid (Sec. III "Boundary Conditions"; Sec. IV, the
boundary-condition study).  The paper's own weight tensors are not
available, so this study uses seeded Gaussian layers of the paper's channel
count, c_in = c_out = 16, 3x3, N(0, 1/(9*16)):

* the periodic spectrum is the union of the symbols' singular values
  (``lfa_svd``), sorted descending;
* the Dirichlet spectrum is that of the dense zero-padded operator
  (``dirichlet_operator``, LAPACK), sorted descending;
* the gap is |sigma_D(i) - sigma_P(i)| / sigma_P(0), index by index over all
  n*n*16 values: reported as its maximum and mean, with the ratio of the
  two largest singular values.

Run ``python -m oracle.boundary_study [n ...]`` (default 4 8 16; the dense
SVD of n = 32 is a 16384 x 16384 matrix: minutes and 2 GiB of host memory).
"""

from __future__ import annotations

import sys

import numpy as np

from .lfa64 import dirichlet_operator, lfa_svd


def layer(n: int, seed: int, c: int = 16, k: int = 3):
    """W [c, c, k, k] of N(0, 1/(k*k*c)) values, float64, seeded (the same
    draw as the tests' random layers)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((c, c, k, k)) * np.sqrt(1.0 / (k * k * c))


def boundary_gap(W, n: int):
    """Gap between the sorted periodic and zero-padded spectra of W on the
    n x n grid: dict(max, mean, top_ratio) relative to sigma_P(0)."""
    sp = np.sort(lfa_svd(W, n, n).ravel())[::-1]
    sd = np.linalg.svd(dirichlet_operator(W, n, n), compute_uv=False)
    g = np.abs(sd - sp) / sp[0]
    return dict(max=float(g.max()), mean=float(g.mean()), top_ratio=float(sd[0] / sp[0]))


def study(sizes=(4, 8, 16), seeds=(41, 42, 43)):
    """{n: dict(max, mean, top_ratio)} averaged over the seeds."""
    out = {}
    for n in sizes:
        rows = [boundary_gap(layer(n, s), n) for s in seeds]
        out[n] = {key: float(np.mean([r[key] for r in rows])) for key in rows[0]}
    return out


def main(argv=None):
    sizes = tuple(int(a) for a in (argv if argv else sys.argv[1:])) or (4, 8, 16)
    print("n     max gap   mean gap  sigma_max(D)/sigma_max(P)   (c = 16, 3x3, mean of 3 seeds)")
    for n, r in study(sizes).items():
        print(f"{n:<5d} {r['max']:.4f}    {r['mean']:.4f}    {r['top_ratio']:.4f}", flush=True)


if __name__ == "__main__":
    main()
