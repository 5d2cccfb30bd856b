"""Pins of the FP64 oracle against what the paper and the mathematics fix.

No GPU.  Each test names the oracle function it pins and the passage (or the
mathematical fact) that fixes the expected value.  Expected values never come
from the oracle's own formulas: they come from brute force on an operator
built independently (torch's circular conv2d), closed forms, invariants, the
FFT identity, finite differences, or fixtures under tests/golden/.
"""

import os

import numpy as np
import pytest
import torch

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def torch_circular_operator(W, n, m):
    """The periodic convolution unrolled by running torch's conv2d on every
    basis vector of a circularly padded input: an implementation of
    (A*f)(x) = sum_y M_y f(x+y) that shares nothing with the oracle.
    Indexing matches the oracle: (x1*m + x2)*c + channel."""
    W = torch.as_tensor(np.asarray(W, dtype=np.float64))
    c_out, c_in, kh, kw = W.shape
    N = n * m * c_in
    eye = torch.eye(N, dtype=torch.float64).reshape(N, n, m, c_in).permute(0, 3, 1, 2)
    pad = ((kw - 1) // 2, kw // 2, (kh - 1) // 2, kh // 2)
    # circular padding wraps at most once: fine while the kernel fits the grid
    x = torch.nn.functional.pad(eye, pad, mode="circular")
    y = torch.nn.functional.conv2d(x, W)                       # (N, c_out, n, m)
    cols = y.permute(0, 2, 3, 1).reshape(N, n * m * c_out)     # column per basis vector
    return cols.T.numpy()


def torch_zero_padded_operator(W, n, m):
    W = torch.as_tensor(np.asarray(W, dtype=np.float64))
    c_out, c_in, kh, kw = W.shape
    N = n * m * c_in
    eye = torch.eye(N, dtype=torch.float64).reshape(N, n, m, c_in).permute(0, 3, 1, 2)
    pad = ((kw - 1) // 2, kw // 2, (kh - 1) // 2, kh // 2)
    x = torch.nn.functional.pad(eye, pad, mode="constant", value=0.0)
    y = torch.nn.functional.conv2d(x, W)
    return y.permute(0, 2, 3, 1).reshape(N, n * m * c_out).T.numpy()


BRUTE_CASES = [
    # c_out, c_in, kh, kw, n, m
    (4, 4, 3, 3, 8, 8),
    (3, 2, 3, 3, 6, 5),
    (2, 4, 3, 3, 4, 7),
    (4, 4, 1, 1, 5, 5),
    (2, 3, 5, 5, 6, 6),
    (3, 3, 3, 5, 5, 7),
    (2, 2, 2, 2, 4, 4),       # even kernel: centred at (k-1)//2
    (1, 1, 3, 3, 8, 8),
]


# --- P1: brute force --------------------------------------------------------

@pytest.mark.parametrize("case", BRUTE_CASES)
def test_unrolled_operator_matches_torch_conv2d(case):
    """oracle.unrolled_operator == torch circular conv2d, entry by entry
    (definition of the operator, Sec. III "Convolutional Mappings")."""
    c_out, c_in, kh, kw, n, m = case
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=11, dtype=np.float64)
    np.testing.assert_array_equal(oracle.unrolled_operator(W, n, m), torch_circular_operator(W, n, m))


@pytest.mark.parametrize("case", BRUTE_CASES)
def test_brute_force_singular_values(case):
    """Union over frequencies of the symbol singular values == singular values
    of the dense unrolled operator (Sec. III "Convolution Theorem": the Fourier
    modes make the operator block diagonal).  Dense SVD by LAPACK dgesdd of
    the torch-built matrix."""
    c_out, c_in, kh, kw, n, m = case
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=7, dtype=np.float64)
    dense = torch_circular_operator(W, n, m)
    s_dense = np.sort(np.linalg.svd(dense, compute_uv=False))[::-1]
    s_lfa = np.sort(oracle.lfa_svd(W, n, m).ravel())[::-1]
    # the dense operator has n*m*max(c) - n*m*min(c) extra zero singular values
    # only when it is not square: compare the nonzero part and count
    r = min(c_out, c_in)
    assert s_lfa.size == n * m * r
    np.testing.assert_allclose(s_lfa, s_dense[: s_lfa.size], rtol=0, atol=1e-13 * s_dense[0])
    assert np.all(s_dense[s_lfa.size:] <= 1e-13 * s_dense[0])


def test_brute_force_config_n8_c4():
    """The 4->4 channel, 8x8 grid brute-force workload: dense 256x256."""
    L, W = workloads.brute_force_small()
    dense = torch_circular_operator(W, L.n, L.m)
    assert dense.shape == (256, 256)
    s_dense = np.sort(np.linalg.svd(dense, compute_uv=False))[::-1]
    s_lfa = np.sort(oracle.lfa_svd(W, L.n, L.m).ravel())[::-1]
    np.testing.assert_allclose(s_lfa, s_dense, rtol=0, atol=1e-13 * s_dense[0])


def test_dirichlet_operator_matches_torch_zero_padding():
    """oracle.dirichlet_operator == torch conv2d with zero padding (Sec. III
    "Boundary Conditions")."""
    _, W = workloads.random_layer(3, 2, 3, 3, 5, 6, seed=5, dtype=np.float64)
    np.testing.assert_array_equal(oracle.dirichlet_operator(W, 5, 6), torch_zero_padded_operator(W, 5, 6))


# --- Convolution theorem / symbol sign -------------------------------------

@pytest.mark.parametrize("n,m", [(5, 6), (4, 4), (1, 3), (7, 2)])
def test_frequency_grid_is_the_dft_dual_grid(n, m):
    """oracle.frequency_grid (Algorithm 1, Init; the dual torus of Sec. III):
    the characters e^{-2 pi i <k, x>} over its frequencies are exactly the
    rows of numpy's 2-D DFT of the unit impulses on the n x m torus, in the
    same (p, q) order, and they are n m distinct, mutually orthogonal modes."""
    k = oracle.frequency_grid(n, m)
    assert k.shape == (n, m, 2)
    x1, x2 = np.meshgrid(np.arange(n), np.arange(m), indexing="ij")
    chars = np.exp(-2j * np.pi * (k[..., 0, None, None] * x1 + k[..., 1, None, None] * x2))
    impulses = np.eye(n * m).reshape(n * m, n, m)                 # impulse at (x1, x2)
    dft = np.fft.fft2(impulses, axes=(-2, -1))                    # [x][p][q]
    expect = np.transpose(dft.reshape(n, m, n, m), (2, 3, 0, 1))  # [p][q][x1][x2]
    np.testing.assert_allclose(chars, expect, atol=1e-12)
    E = chars.reshape(n * m, n * m)
    np.testing.assert_allclose(E @ E.conj().T, n * m * np.eye(n * m), atol=1e-11)
    # every frequency lies in [0, 1)^2 (one representative per class)
    assert np.all(k >= 0) and np.all(k < 1)


def test_fourier_mode_is_invariant_subspace():
    """(A*f_k)(x) = A_k f_k(x) for f_k = e^{2 pi i <k,x>} v (Sec. III
    "Convolution Theorem"): apply the torch-built operator to a Fourier mode
    and read off the symbol.  Pins the +2 pi i sign and the tap centring."""
    c_out, c_in, kh, kw, n, m = 3, 2, 3, 3, 6, 5
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=3, dtype=np.float64)
    dense = torch_circular_operator(W, n, m)
    A = oracle.symbols(W, n, m)
    x1, x2 = np.meshgrid(np.arange(n), np.arange(m), indexing="ij")
    rng = np.random.default_rng(0)
    for p, q in [(0, 0), (1, 2), (5, 4), (3, 1)]:
        v = rng.standard_normal(c_in) + 1j * rng.standard_normal(c_in)
        wave = np.exp(2j * np.pi * (p * x1 / n + q * x2 / m)).ravel()
        f = np.kron(wave, v)
        g = dense @ f
        expect = np.kron(wave, A[p, q] @ v)
        np.testing.assert_allclose(g, expect, atol=1e-13)


def test_shift_symbol_golden():
    """Single tap at offset (1,0): symbol i^p on a 4x4 grid (golden fixture)."""
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 2, 1] = 1.0
    A = oracle.symbols(W, 4, 4)[:, :, 0, 0]
    for p, q, re, im in _load("shift_symbol_4x4.txt"):
        assert abs(A[int(p), int(q)] - (re + 1j * im)) < 1e-15


def test_laplacian_golden_and_closed_form():
    """P4: single channel, 5-point Laplacian stencil: sigma = |4 - 2cos t1 - 2cos t2|."""
    lap = np.array([[0, -1, 0], [-1, 4, -1], [0, -1, 0]], dtype=np.float64)[None, None]
    s = oracle.lfa_svd(lap, 4, 4)[:, :, 0]
    np.testing.assert_allclose(s, _load("laplacian_symbol_4x4.txt"), atol=1e-14)
    n, m = 16, 12
    s = oracle.lfa_svd(lap, n, m)[:, :, 0]
    t1 = 2 * np.pi * np.arange(n)[:, None] / n
    t2 = 2 * np.pi * np.arange(m)[None, :] / m
    np.testing.assert_allclose(s, np.abs(4 - 2 * np.cos(t1) - 2 * np.cos(t2)), atol=1e-14)


# --- P5: FFT identity -------------------------------------------------------

@pytest.mark.parametrize("case", [(3, 2, 3, 3, 8, 6), (5, 5, 7, 7, 9, 9), (2, 3, 1, 1, 4, 4)])
def test_fft_identity(case):
    """A_k(p,q) = n*m * ifft2(kernel scattered to (y mod n, y mod m))[p,q]: the
    mathematics behind the FFT method the paper compares with (Sec. I, Sec. II)."""
    c_out, c_in, kh, kw, n, m = case
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=9, dtype=np.float64)
    K = np.zeros((c_out, c_in, n, m))
    for a in range(kh):
        for b in range(kw):
            K[:, :, (a - (kh - 1) // 2) % n, (b - (kw - 1) // 2) % m] += W[:, :, a, b]
    A_fft = n * m * np.fft.ifft2(K, axes=(2, 3))          # (c_out, c_in, n, m)
    A = oracle.symbols(W, n, m)
    np.testing.assert_allclose(A, np.transpose(A_fft, (2, 3, 0, 1)), atol=1e-14)


def test_sampled_frequencies_match_full_grid():
    """symbols(freqs=...) picks the same entries as the full grid."""
    _, W = workloads.random_layer(3, 4, 3, 3, 7, 9, seed=2, dtype=np.float64)
    A = oracle.symbols(W, 7, 9)
    fr = np.array([[0, 0], [6, 8], [3, 2], [1, 7]])
    np.testing.assert_array_equal(oracle.symbols(W, 7, 9, fr), A[fr[:, 0], fr[:, 1]])


# --- P2: Parseval ----------------------------------------------------------

@pytest.mark.parametrize("case", [(16, 16, 3, 3, 32, 32), (8, 5, 3, 3, 6, 10), (4, 9, 5, 5, 7, 7)])
def test_parseval(case):
    """sum sigma^2 = n*m*||W||_F^2 (no tap aliasing): trace of A^H A summed over
    the Fourier basis equals the Frobenius norm of the unrolled operator."""
    c_out, c_in, kh, kw, n, m = case
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=4, dtype=np.float64)
    s = oracle.lfa_svd(W, n, m)
    np.testing.assert_allclose(np.sum(s**2), n * m * np.sum(W**2), rtol=1e-13)


# --- P3: identity / orthogonal tap ------------------------------------------

def test_identity_kernel_all_ones():
    c = 5
    W = np.zeros((c, c, 3, 3))
    W[:, :, 1, 1] = np.eye(c)
    np.testing.assert_allclose(oracle.lfa_svd(W, 6, 6), 1.0, atol=1e-15)


def test_orthogonal_offcentre_tap_all_ones():
    """Single off-centre tap holding an orthogonal Q: the operator is a shift
    (a permutation) tensor Q, so every singular value is 1."""
    c = 6
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((c, c)))
    W = np.zeros((c, c, 3, 3))
    W[:, :, 0, 2] = Q
    np.testing.assert_allclose(oracle.lfa_svd(W, 5, 7), 1.0, atol=1e-14)


# --- P6, P7: symmetries and invariances --------------------------------------

def test_conjugate_symmetry():
    """Real W: A_{-k} = conj(A_k), so sigma(k) = sigma(-k)."""
    n, m = 8, 6
    _, W = workloads.random_layer(4, 3, 3, 3, n, m, seed=6, dtype=np.float64)
    A = oracle.symbols(W, n, m)
    neg = A[(-np.arange(n)) % n][:, (-np.arange(m)) % m]
    np.testing.assert_allclose(neg, np.conj(A), atol=1e-15)


def test_invariances():
    n = 6
    _, W = workloads.random_layer(5, 4, 3, 3, n, n, seed=8, dtype=np.float64)
    s = np.sort(oracle.lfa_svd(W, n).ravel())
    # scaling
    np.testing.assert_allclose(np.sort(oracle.lfa_svd(-2.5 * W, n).ravel()), 2.5 * s, rtol=1e-13)
    # common orthogonal transforms of all taps
    rng = np.random.default_rng(2)
    Qo, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    Qi, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    W2 = np.einsum("po,oiab,iq->pqab", Qo, W, Qi)
    np.testing.assert_allclose(np.sort(oracle.lfa_svd(W2, n).ravel()), s, atol=1e-13 * s.max())
    # channel permutation
    W3 = W[rng.permutation(5)][:, rng.permutation(4)]
    np.testing.assert_allclose(np.sort(oracle.lfa_svd(W3, n).ravel()), s, atol=1e-13 * s.max())


# --- P8: rank -----------------------------------------------------------------

def test_rank_one_taps():
    """Rank-one taps: rank A_k <= number of taps, so min(c) - 9 zero sigma."""
    L, W = workloads.rank_one_taps(c_out=24, c_in=16, n=4)
    s = oracle.lfa_svd(W.astype(np.float64), L.n)
    assert s.shape == (4, 4, 16)
    assert np.all(s[:, :, 9:] <= 1e-13 * s[:, :, :1])
    assert np.all(s[:, :, 8] > 1e-6 * s[:, :, 0])


def test_common_vector_closed_form():
    """W_y = c_y a b^T  =>  sigma_1(k) = ||a|| ||b|| |sum_y c_y e^{2 pi i <k,y>}|,
    other singular values zero.  The scalar sum is evaluated with numpy's FFT
    (the FFT identity), not with the oracle."""
    rng = np.random.default_rng(12)
    a, b, cy = rng.standard_normal(6), rng.standard_normal(4), rng.standard_normal((3, 3))
    W = np.einsum("o,i,xy->oixy", a, b, cy)
    n, m = 7, 5
    s = oracle.lfa_svd(W, n, m)
    K = np.zeros((n, m))
    for x in range(3):
        for y in range(3):
            K[(x - 1) % n, (y - 1) % m] += cy[x, y]
    sym = n * m * np.fft.ifft2(K)
    np.testing.assert_allclose(s[:, :, 0], np.linalg.norm(a) * np.linalg.norm(b) * np.abs(sym), rtol=1e-13)
    assert np.all(s[:, :, 1:] <= 1e-13 * s[:, :, :1].max())


# --- P9: count ----------------------------------------------------------------

def test_counts_match_table2():
    """#sigma = n*m*min(c_in, c_out), against the counts printed in Table II."""
    for n, count in _load("table2_sigma_counts.txt"):
        assert workloads.Layer(16, 16, 3, 3, int(n), int(n)).num_sigma == int(count)
    s = oracle.lfa_svd(np.random.default_rng(0).standard_normal((16, 16, 3, 3)), 8, 4)
    assert s.size == 8 * 4 * 16


# --- P10: vectors and lift ------------------------------------------------------

def test_vectors_orthonormal_and_residual():
    _, W = workloads.random_layer(7, 5, 3, 3, 6, 6, seed=13, dtype=np.float64)
    s, U, V = oracle.lfa_svd(W, 6, compute_uv=True)
    A = oracle.symbols(W, 6)
    eye = np.eye(5)
    UhU = np.conj(np.swapaxes(U, -1, -2)) @ U
    VhV = np.conj(np.swapaxes(V, -1, -2)) @ V
    np.testing.assert_allclose(UhU, np.broadcast_to(eye, UhU.shape), atol=1e-13)
    np.testing.assert_allclose(VhV, np.broadcast_to(eye, VhV.shape), atol=1e-13)
    np.testing.assert_allclose(A @ V, U * s[..., None, :], atol=1e-13)
    assert np.all(np.diff(s, axis=-1) <= 0)


def test_lift_gives_global_singular_vectors():
    """U_hat = F^out U, V_hat = F^in V are orthonormal and satisfy
    A V_hat = U_hat S for the torch-built unrolled operator (Sec. III)."""
    n, m = 4, 3
    _, W = workloads.random_layer(3, 2, 3, 3, n, m, seed=21, dtype=np.float64)
    dense = torch_circular_operator(W, n, m)
    s, U, V = oracle.lfa_svd(W, n, m, compute_uv=True)
    Uh_all, Vh_all, s_all = [], [], []
    for p in range(n):
        for q in range(m):
            Uh, Vh = oracle.lift(U[p, q], V[p, q], n, m, p, q)
            np.testing.assert_allclose(dense @ Vh, Uh * s[p, q][None, :], atol=1e-13)
            Uh_all.append(Uh)
            Vh_all.append(Vh)
            s_all.append(s[p, q])
    Vh_all = np.concatenate(Vh_all, axis=1)
    Uh_all = np.concatenate(Uh_all, axis=1)
    np.testing.assert_allclose(np.conj(Vh_all.T) @ Vh_all, np.eye(Vh_all.shape[1]), atol=1e-13)
    np.testing.assert_allclose(np.conj(Uh_all.T) @ Uh_all, np.eye(Uh_all.shape[1]), atol=1e-13)
    assert Vh_all.shape == (n * m * 2, n * m * 2)     # full SVD of the square-in part


# --- P11: gradient --------------------------------------------------------------

def test_sigma_grad_matches_finite_differences():
    n, m = 5, 4
    _, W = workloads.random_layer(4, 3, 3, 3, n, m, seed=17, dtype=np.float64)
    picks = np.array([[1, 2, 0], [3, 1, 2], [0, 0, 1]])
    g = np.array([1.0, -0.5, 2.0])
    dW = oracle.sigma_grad(W, n, m, picks, g)

    def loss(Wx):
        s = oracle.lfa_svd(Wx, n, m)
        return sum(gi * s[p, q, j] for gi, (p, q, j) in zip(g, picks))

    rng = np.random.default_rng(3)
    for _ in range(4):
        D = rng.standard_normal(W.shape)
        h = 1e-6 * np.linalg.norm(W)
        fd = (loss(W + h * D) - loss(W - h * D)) / (2 * h)
        an = np.sum(dW * D)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_sigma_grad_entrywise_fd():
    """Every entry of the gradient of the largest sigma at one frequency."""
    n = 4
    _, W = workloads.random_layer(2, 2, 3, 3, n, n, seed=5, dtype=np.float64)
    picks = np.array([[1, 3, 0]])
    dW = oracle.sigma_grad(W, n, n, picks)
    h = 1e-6
    for idx in np.ndindex(W.shape):
        Wp, Wm = W.copy(), W.copy()
        Wp[idx] += h
        Wm[idx] -= h
        fd = (oracle.lfa_svd(Wp, n)[1, 3, 0] - oracle.lfa_svd(Wm, n)[1, 3, 0]) / (2 * h)
        assert abs(fd - dW[idx]) < 1e-8


# --- top-k -------------------------------------------------------------------------

def test_topk_order_and_ties():
    s = np.zeros((2, 3, 2))
    s[0, 1, 0] = 5.0
    s[1, 2, 1] = 5.0      # tie: (0,1,0) comes first
    s[1, 0, 0] = 7.0
    s[0, 0, 1] = 3.0
    vals, idx = oracle.topk(s, 4)
    np.testing.assert_array_equal(vals, [7.0, 5.0, 5.0, 3.0])
    np.testing.assert_array_equal(idx, [[1, 0, 0], [0, 1, 0], [1, 2, 1], [0, 0, 1]])
    # brute force on random data
    r = np.random.default_rng(4).random((5, 4, 3))
    vals, idx = oracle.topk(r, 8)
    np.testing.assert_array_equal(vals, np.sort(r.ravel())[::-1][:8])
    np.testing.assert_array_equal(r[idx[:, 0], idx[:, 1], idx[:, 2]], vals)


def test_sigma_error_metric():
    ref = np.array([[4.0, 2.0, 0.0], [1.0, 0.5, 0.25]])
    test = ref + np.array([[0.0, 0.04, 0.0], [0.0, 0.0, 0.001]])
    assert oracle.sigma_error(test, ref) == pytest.approx(0.01)


# --- Dirichlet vs periodic (qualitative claim of Sec. IV) -----------------------

def test_dirichlet_spectrum_approaches_periodic():
    """The boundary's influence on the spectrum shrinks as the grid grows
    (Sec. IV, boundary-condition study): the distance between the sorted
    Dirichlet and periodic spectra, relative to sigma_max, decreases with n."""
    _, W = workloads.random_layer(3, 3, 3, 3, 4, 4, seed=1, dtype=np.float64)
    gaps = []
    for n in (4, 8, 12):
        sp = np.sort(oracle.lfa_svd(W, n).ravel())
        sd = np.sort(np.linalg.svd(oracle.dirichlet_operator(W, n), compute_uv=False))
        gaps.append(np.mean(np.abs(sp - sd)) / sp[-1])
    assert gaps[0] > gaps[1] > gaps[2]


# --- spectral functions applied through the per-symbol SVD ------------------

APPLY_CASES = [
    # c_out, c_in, kh, kw, n, m, batch
    (3, 2, 3, 3, 5, 4, 2),
    (2, 4, 3, 3, 4, 6, 1),
    (4, 4, 3, 3, 6, 6, 3),
    (2, 2, 2, 2, 4, 5, 2),     # even kernel
]


@pytest.mark.parametrize("case", APPLY_CASES)
def test_apply_identity_is_the_convolution(case):
    """oracle.apply_spectral with f(sigma) = sigma is the operator itself:
    torch's conv2d on a circularly padded input (the periodic cross-correlation
    of Sec. III "Convolutional Mappings"), which shares nothing with the
    oracle's transforms."""
    c_out, c_in, kh, kw, n, m, B = case
    rng = np.random.default_rng(31)
    W = rng.standard_normal((c_out, c_in, kh, kw))
    x = rng.standard_normal((B, c_in, n, m))
    pad = ((kw - 1) // 2, kw // 2, (kh - 1) // 2, kh // 2)
    xt = torch.nn.functional.pad(torch.from_numpy(x), pad, mode="circular")
    ref = torch.nn.functional.conv2d(xt, torch.from_numpy(W)).numpy()
    got = oracle.apply_spectral(W, x, n, m, "identity")
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", APPLY_CASES)
@pytest.mark.parametrize("kind", ["pinv", "clip", "truncate"])
def test_apply_spectral_matches_dense_svd(case, kind):
    """Pseudo-inverse, clipping and low-rank truncation through the per-symbol
    SVD equal the same spectral function of the dense operator's SVD (torch's
    circular operator -> numpy.linalg.svd): A^+ = V f(S) U^T, clipped or
    truncated A = U f(S) V^T.  The
    cut-off / clip level lies midway in a gap of the singular values near
    their median (a level on a singular value would make the result depend
    on rounding)."""
    c_out, c_in, kh, kw, n, m, B = case
    rng = np.random.default_rng(32)
    W = rng.standard_normal((c_out, c_in, kh, kw))
    A = torch_circular_operator(W, n, m)
    Ud, Sd, Vdh = np.linalg.svd(A)
    s = np.sort(Sd)
    gaps = np.where(np.diff(s) > 1e-3 * s[-1])[0]
    i = gaps[np.argmin(np.abs(gaps - s.size // 2))]
    level = 0.5 * (s[i] + s[i + 1])
    f = oracle.spectral_factor(Sd, kind, level)
    if kind == "pinv":
        assert np.all(f[Sd > level] == 1.0 / Sd[Sd > level]) and np.all(f[Sd <= level] == 0)
    elif kind == "clip":
        assert np.all(f == np.minimum(Sd, level))
    else:
        assert np.all(f[Sd > level] == Sd[Sd > level]) and np.all(f[Sd <= level] == 0)
    r = Sd.size
    if kind == "pinv":
        x = rng.standard_normal((B, c_out, n, m))
        op = Vdh[:r].T @ np.diag(f) @ Ud[:, :r].T
        c_y = c_in
    else:
        x = rng.standard_normal((B, c_in, n, m))
        op = Ud[:, :r] @ np.diag(f) @ Vdh[:r]
        c_y = c_out
    xv = np.transpose(x, (0, 2, 3, 1)).reshape(B, -1)
    ref = np.transpose((xv @ op.T).reshape(B, n, m, c_y), (0, 3, 1, 2))
    got = oracle.apply_spectral(W, x, n, m, kind, level)
    assert np.max(np.abs(got - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))
    dense = oracle.apply_spectral_dense(W, x, n, m, kind, level)
    assert np.max(np.abs(dense - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))
    if kind == "pinv":
        # Moore-Penrose with the truncated spectrum: A A^+ A = A_kept, and
        # A^+ A A^+ = A^+
        assert np.allclose(op @ A @ op, op, atol=1e-10 * np.abs(op).max())
    if kind == "truncate":
        # Eckart-Young: the kept part has rank #(sigma > level) and leaves a
        # remainder of spectral norm max(sigma <= level)
        kept = int(np.sum(Sd > level))
        assert np.linalg.matrix_rank(op, tol=1e-9 * Sd.max()) == kept
        assert abs(np.linalg.norm(A - op, 2) - Sd[Sd <= level].max()) <= 1e-10 * Sd.max()


def test_apply_pinv_inverts_full_rank_and_clip_above_max_is_identity():
    """For a square operator with every singular value kept, the pseudo-inverse
    undoes the operator (A^+ A x = x); clipping at or above sigma_max changes
    nothing, nor does truncating below sigma_min, while truncating at
    sigma_max leaves nothing."""
    rng = np.random.default_rng(33)
    W = rng.standard_normal((3, 3, 3, 3))
    n, m = 6, 5
    x = rng.standard_normal((2, 3, n, m))
    Ax = oracle.apply_spectral(W, x, n, m, "identity")
    S = oracle.lfa_svd(W, n, m)
    assert S.min() > 1e-3 * S.max()
    back = oracle.apply_spectral(W, Ax, n, m, "pinv", 0.0)
    assert np.max(np.abs(back - x)) <= 1e-12 * np.max(np.abs(x)) * S.max() / S.min()
    same = oracle.apply_spectral(W, x, n, m, "clip", S.max() * (1 + 1e-12))
    assert np.max(np.abs(same - Ax)) <= 1e-12 * np.max(np.abs(Ax))
    # truncation below sigma_min keeps the operator; at or above sigma_max
    # it removes everything
    keep = oracle.apply_spectral(W, x, n, m, "truncate", 0.5 * S.min())
    assert np.max(np.abs(keep - Ax)) <= 1e-12 * np.max(np.abs(Ax))
    gone = oracle.apply_spectral(W, x, n, m, "truncate", S.max())
    assert np.max(np.abs(gone)) == 0.0


# --- strided convolutions as crystals -------------------------------------------

def torch_strided_operator(W, n, m, s):
    """The stride-s periodic convolution unrolled with torch: circular padding
    as for stride 1, then conv2d with stride s, on every basis vector."""
    W = torch.as_tensor(np.asarray(W, dtype=np.float64))
    c_out, c_in, kh, kw = W.shape
    N = n * m * c_in
    eye = torch.eye(N, dtype=torch.float64).reshape(N, n, m, c_in).permute(0, 3, 1, 2)
    pad = ((kw - 1) // 2, kw // 2, (kh - 1) // 2, kh // 2)
    y = torch.nn.functional.conv2d(torch.nn.functional.pad(eye, pad, mode="circular"), W, stride=s)
    assert tuple(y.shape[2:]) == (n // s, m // s)
    return y.permute(0, 2, 3, 1).reshape(N, -1).T.numpy()


STRIDED_CASES = [
    # c_out, c_in, kh, kw, n, m, s
    (3, 2, 3, 3, 8, 6, 2),
    (2, 3, 3, 3, 6, 6, 3),
    (4, 1, 7, 7, 8, 8, 2),      # stem-like 7x7, stride 2
    (3, 2, 1, 1, 6, 4, 2),      # 1x1 shortcut, stride 2
    (2, 2, 2, 4, 8, 8, 2),      # even extents
    (2, 3, 3, 3, 5, 4, 1),      # stride 1
]


@pytest.mark.parametrize("case", STRIDED_CASES)
def test_strided_operator_matches_torch(case):
    c_out, c_in, kh, kw, n, m, s = case
    W = np.random.default_rng(51).standard_normal((c_out, c_in, kh, kw))
    np.testing.assert_allclose(oracle.strided_operator(W, n, m, s), torch_strided_operator(W, n, m, s),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("case", STRIDED_CASES)
def test_crystal_symbols_brute_force_and_modes(case):
    """The singular values of the crystal symbols are those of the dense
    strided operator (brute force), their count is (n/s)(m/s) min(c_out,
    s^2 c_in), and the operator maps each crystal Fourier mode to the mode
    of the same frequency on the output torus with coefficients A_k v: this
    fixes the phase convention and the column order of the symbol."""
    c_out, c_in, kh, kw, n, m, s = case
    rng = np.random.default_rng(52)
    W = rng.standard_normal((c_out, c_in, kh, kw))
    A = oracle.crystal_symbols(W, n, m, s)
    nc, mc = n // s, m // s
    assert A.shape == (nc, mc, c_out, s * s * c_in)
    S = np.linalg.svd(A, compute_uv=False)
    D = oracle.strided_operator(W, n, m, s)
    Sd = np.linalg.svd(D, compute_uv=False)
    r = min(c_out, s * s * c_in)
    assert S.size == nc * mc * r == min(D.shape)
    np.testing.assert_allclose(np.sort(S.ravel()), np.sort(Sd), rtol=0, atol=1e-12 * Sd.max())
    # modes: f(s X + d)[i] = e^{2 pi i <k, X>} v[i s^2 + d1 s + d2]
    for (p, q) in [(0, 0), (1, 0), (nc - 1, mc - 1), (nc // 2, 1 % mc)]:
        v = rng.standard_normal(s * s * c_in) + 1j * rng.standard_normal(s * s * c_in)
        f = np.zeros((n, m, c_in), dtype=np.complex128)
        for z1 in range(n):
            for z2 in range(m):
                X1, d1 = divmod(z1, s)
                X2, d2 = divmod(z2, s)
                ph = np.exp(2j * np.pi * (p * X1 / nc + q * X2 / mc))
                f[z1, z2, :] = ph * v[np.arange(c_in) * s * s + d1 * s + d2]
        y = (D @ f.ravel()).reshape(nc, mc, c_out)
        x1, x2 = np.meshgrid(np.arange(nc), np.arange(mc), indexing="ij")
        want = np.exp(2j * np.pi * (p * x1 / nc + q * x2 / mc))[:, :, None] * (A[p, q] @ v)[None, None, :]
        assert np.max(np.abs(y - want)) <= 1e-12 * np.max(np.abs(want))


def test_crystal_symbols_stride_one_and_parseval():
    """Stride 1 gives the ordinary symbols; for any stride, sum sigma^2 =
    (n/s)(m/s) ||W||_F^2 while the kernel fits the grid (every output point
    reads each tap once, at distinct input points)."""
    rng = np.random.default_rng(53)
    W = rng.standard_normal((4, 3, 3, 3))
    np.testing.assert_allclose(oracle.crystal_symbols(W, 6, 5, 1), oracle.symbols(W, 6, 5), rtol=0, atol=1e-14)
    for (n, m, s) in [(8, 8, 2), (9, 6, 3), (8, 4, 4)]:
        S = np.linalg.svd(oracle.crystal_symbols(W, n, m, s), compute_uv=False)
        total = (n // s) * (m // s) * np.sum(W ** 2)
        assert abs(np.sum(S ** 2) - total) <= 1e-12 * total


def test_boundary_study_c16_gap_shrinks_with_the_grid():
    """The paper's boundary-condition study at its channel count (c = 16,
    3x3; Sec. III "Boundary Conditions", Sec. IV): the sorted periodic (LFA)
    and zero-padded spectra of the same seeded layers differ by a gap that
    shrinks with the grid -- about halving from n = 4 to n = 8, as the
    share of grid points next to the boundary halves -- and the largest
    singular values approach each other (oracle.boundary_study)."""
    from oracle import boundary_study as bs

    r = bs.study(sizes=(4, 8), seeds=(41, 42))
    assert r[8]["max"] < r[4]["max"] and r[8]["mean"] < r[4]["mean"]
    assert 0.35 <= r[8]["mean"] / r[4]["mean"] <= 0.65, r
    assert abs(1 - r[8]["top_ratio"]) < abs(1 - r[4]["top_ratio"]), r
    # zero padding is the periodic convolution on the (n+2)-torus restricted
    # to an n x n block (3x3 taps reach one cell past the block, which holds
    # zeros): an isometric compression, so its largest singular value is at
    # most that torus's largest symbol singular value
    for n in (4, 8):
        W = bs.layer(n, 41)
        sd = np.linalg.svd(oracle.dirichlet_operator(W, n, n), compute_uv=False)
        assert sd[0] <= oracle.lfa_svd(W, n + 2, n + 2).max() * (1 + 1e-12)


# --- Phase normalisation of the singular pairs ----------------------------

def test_phase_normalize_hand_examples():
    """oracle.phase_normalize on pairs whose answer is written out by hand:
    the entry of largest modulus of v becomes real positive, u takes the
    same factor, the lowest row wins an exact tie, and with V absent the
    rule applies to u."""
    s = 1 / np.sqrt(2)
    # already normalised: the largest entry (0.8, row 1) is real positive
    U, V = oracle.phase_normalize(np.array([[1j]]), np.array([[0.6j], [0.8]]))
    np.testing.assert_allclose(V, [[0.6j], [0.8]], atol=1e-15)
    np.testing.assert_allclose(U, [[1j]], atol=1e-15)
    # largest entry 0.8i (row 0): the factor is -i
    U, V = oracle.phase_normalize(np.array([[1.0]]), np.array([[0.8j], [0.6]]))
    np.testing.assert_allclose(V, [[0.8], [-0.6j]], atol=1e-15)
    np.testing.assert_allclose(U, [[-1j]], atol=1e-15)
    # exact tie |i/sqrt2| = |1/sqrt2|: row 0 decides, factor -i
    _, V = oracle.phase_normalize(None, np.array([[1j * s], [s]]))
    np.testing.assert_allclose(V, [[s], [-1j * s]], atol=1e-15)
    # U alone: the largest entry -2 (row 0) becomes 2
    U, V = oracle.phase_normalize(np.array([[-2.0], [1.0]]), None)
    assert V is None
    np.testing.assert_allclose(U, [[2.0], [-1.0]], atol=1e-15)
    # two columns normalised independently
    _, V = oracle.phase_normalize(None, np.array([[1j, 0.1], [0.1, -3.0]]))
    np.testing.assert_allclose(V, [[1, 0.1 * -1], [-0.1j, 3.0]], atol=1e-15)


def test_phase_normalize_removes_the_gauge():
    """Any SVD of a matrix with simple singular values differs from another
    by one phase per pair (U D, V D with D diagonal unitary).  After
    oracle.phase_normalize two such SVDs are the same, the factorisation
    A = U diag(s) V^H still holds, every largest entry of v_j is real
    positive, and a second normalisation changes nothing."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 7, 5)) + 1j * rng.standard_normal((4, 7, 5))
    s, U, V = oracle.svd_symbols(A)
    D = np.exp(2j * np.pi * rng.random((4, 1, 5)))
    U1, V1 = oracle.phase_normalize(U, V)
    U2, V2 = oracle.phase_normalize(U * D, V * D)
    np.testing.assert_allclose(U1, U2, atol=1e-12)
    np.testing.assert_allclose(V1, V2, atol=1e-12)
    np.testing.assert_allclose((U1 * s[:, None, :]) @ np.conj(np.swapaxes(V1, -1, -2)), A, atol=1e-12)
    top = np.take_along_axis(V1, np.argmax(np.abs(V1), axis=1)[:, None, :], axis=1)
    assert np.all(top.real > 0) and np.all(np.abs(top.imag) <= 1e-15 * top.real)
    U3, V3 = oracle.phase_normalize(U1, V1)
    np.testing.assert_allclose(U3, U1, atol=1e-15)
    np.testing.assert_allclose(V3, V1, atol=1e-15)
