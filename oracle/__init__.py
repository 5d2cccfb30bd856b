"""FP64 CPU oracle for the LFA singular value decomposition of a periodic,
stride-1, multi-channel 2-D convolution.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library in ``paper_2506_05617_amd``.

Everything here follows the paper's definitions directly, in float64 /
complex128, with NumPy/LAPACK as the only library primitives:

* ``frequency_grid``   -- the dual torus of frequencies (Sec. III,
  "Convolution Theorem"; Algorithm 1, Init step).
* ``tap_offsets``      -- kernel taps as offsets y of a neighbourhood centred
  at x (Sec. III, "Convolutional Mappings in CNNs", stencil figure).
* ``symbols``          -- the c_out x c_in symbol A_k = sum_y M_y e^{2 pi i <k,y>}
  (Sec. III, "Convolution Theorem"; Algorithm 1, symbol step).
* ``svd_symbols``      -- per-frequency SVD A_k = U_k S_k V_k^* (Sec. III,
  "Convolution Theorem"; Algorithm 1, SVD step) via ``numpy.linalg.svd``.
* ``phase_normalize``  -- the common phase of each singular pair fixed so that
  the largest-modulus entry of v_j is real and positive (post-processing of
  the SVD step; a convention, the paper leaves the phase open).
* ``unrolled_operator``-- the dense matrix of (A*f)(x) = sum_y M_y f(x+y) on the
  periodic torus (Sec. I matrix view; Sec. III "Convolutional Mappings").
* ``lift``             -- global singular vectors F_k U_k, F_k V_k (Sec. III,
  "Convolution Theorem").
* ``sigma_grad``       -- gradient of a sum of selected singular values with
  respect to the weights (first-order perturbation of a simple singular value;
  not in the paper, used for the spectral-norm regularisation it motivates,
  Sec. II "Application Domains").
* ``topk``             -- k largest singular values of a layer with a fixed
  tie order.
* ``dirichlet_operator`` -- the zero-padded (Dirichlet) operator the paper
  compares against (Sec. III "Boundary Conditions"; Sec. IV).
* ``strided_operator``, ``crystal_symbols`` -- a stride-s convolution as a
  map between crystal tori: the input has s*s*c_in points per cell of the
  coarse lattice (Sec. III "Introduction to Lattices and Crystals").
* ``apply_spectral``   -- ``y = U f(Sigma) V^* x`` for the identity, a
  pseudo-inverse or singular-value clipping, through the per-symbol SVD
  (Sec. III "Convolution Theorem": the global SVD is the lift of the
  symbols' SVDs); ``apply_spectral_dense`` is the same from the SVD of the
  unrolled operator.

Parity pins: every function above is pinned by tests in
``tests/test_oracle_pins.py`` against brute force, closed forms, invariants,
or values printed in the paper (``tests/golden/``).
"""

from .lfa64 import (  # noqa: F401
    frequency_grid,
    tap_offsets,
    phase_factors,
    symbols,
    svd_symbols,
    phase_normalize,
    lfa_svd,
    unrolled_operator,
    dirichlet_operator,
    strided_operator,
    crystal_symbols,
    fourier_basis,
    lift,
    spectral_factor,
    apply_spectral,
    apply_spectral_dense,
    sigma_grad,
    topk,
    sigma_error,
)
