"""Plain, slow, float64 implementation of the LFA SVD of a periodic convolution.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Shares no code with
the HIP library.

Conventions (each one a reading of the paper, listed in the design notes):

* A weight tensor is PyTorch channel-first ``W[c_out, c_in, kh, kw]`` (Sec. IV,
  "Runtime Analysis": the implementation operates on PyTorch convolution
  weights stored channel-first).  Tap ``(a, b)`` is the matrix
  ``M_y = W[:, :, a, b]`` (size c_out x c_in, Sec. III "Convolutional
  Mappings") at offset ``y = (a - (kh-1)//2, b - (kw-1)//2)``: the
  neighbourhood is centred at x (stencil figure, Sec. III).
* The operator is ``(A*f)(x) = sum_y M_y f(x + y)`` on the periodic n x m torus
  (Sec. III "Convolutional Mappings"), i.e. a cross-correlation, which is what
  ``torch.nn.functional.conv2d`` computes on a circularly padded input.
* The first spatial axis has length n and frequencies ``p/n``; the second has
  length m and frequencies ``q/m`` (Algorithm 1, Init: X uses 1/n, Y uses 1/m).
* The symbol uses the ``+2 pi i`` sign of the paper (Sec. III "Convolution
  Theorem"; Algorithm 1 symbol step).
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Grid and taps
# ---------------------------------------------------------------------------

def frequency_grid(n: int, m: int) -> np.ndarray:
    """Frequencies of the dual torus T*_{n,m} (Sec. III "Convolution Theorem";
    Algorithm 1 Init): ``k = (p/n, q/m)`` for ``0 <= p < n``, ``0 <= q < m``.

    Returns an ``(n, m, 2)`` float64 array of k (not 2*pi*k).
    """
    p = np.arange(n, dtype=np.float64) / n
    q = np.arange(m, dtype=np.float64) / m
    k = np.empty((n, m, 2), dtype=np.float64)
    k[:, :, 0] = p[:, None]
    k[:, :, 1] = q[None, :]
    return k


def tap_offsets(kh: int, kw: int) -> np.ndarray:
    """Offsets y of the kernel taps, neighbourhood centred at x (Sec. III,
    stencil figure).  Returns ``(kh, kw, 2)`` int64: ``y = (a - (kh-1)//2,
    b - (kw-1)//2)`` for tap ``(a, b)``."""
    y = np.empty((kh, kw, 2), dtype=np.int64)
    y[:, :, 0] = (np.arange(kh) - (kh - 1) // 2)[:, None]
    y[:, :, 1] = (np.arange(kw) - (kw - 1) // 2)[None, :]
    return y


def phase_factors(n: int, m: int, kh: int, kw: int, freqs=None) -> np.ndarray:
    """``e^{2 pi i <k, y>}`` for every requested frequency and tap.

    The integer product ``p*y1`` is reduced modulo n (and ``q*y2`` modulo m)
    before the angle is formed, so the angle is exact up to one rounding.
    ``freqs`` is an optional ``(F, 2)`` integer array of ``(p, q)``; by default
    all ``n*m`` frequencies in row-major ``(p, q)`` order.
    Returns ``(F, kh, kw)`` complex128.
    """
    if freqs is None:
        pp, qq = np.meshgrid(np.arange(n), np.arange(m), indexing="ij")
        freqs = np.stack([pp.ravel(), qq.ravel()], axis=1)
    freqs = np.asarray(freqs, dtype=np.int64)
    y = tap_offsets(kh, kw)
    rp = np.mod(freqs[:, 0, None, None] * y[None, :, :, 0], n)
    rq = np.mod(freqs[:, 1, None, None] * y[None, :, :, 1], m)
    ang = 2.0 * np.pi * (rp / n + rq / m)
    return np.exp(1j * ang)


# ---------------------------------------------------------------------------
# Symbols and their SVD
# ---------------------------------------------------------------------------

def symbols(W, n: int, m: int | None = None, freqs=None) -> np.ndarray:
    """Symbol ``A_k = sum_{y in N} M_y e^{2 pi i <k, y>}`` (Sec. III
    "Convolution Theorem"; Algorithm 1 symbol step), by direct summation over
    the taps.

    ``W``: real ``[c_out, c_in, kh, kw]`` (any float dtype; upcast to float64).
    Returns ``[n, m, c_out, c_in]`` complex128 (row-major, the layout the paper
    keeps, Sec. IV "Memory Layout Effects"), or ``[F, c_out, c_in]`` when
    ``freqs`` lists F frequencies ``(p, q)``.
    """
    m = n if m is None else m
    W = np.asarray(W, dtype=np.float64)
    c_out, c_in, kh, kw = W.shape
    ph = phase_factors(n, m, kh, kw, freqs)            # (F, kh, kw)
    F = ph.shape[0]
    A = np.zeros((F, c_out, c_in), dtype=np.complex128)
    for a in range(kh):
        for b in range(kw):
            A += ph[:, a, b, None, None] * W[None, :, :, a, b]
    if freqs is None:
        A = A.reshape(n, m, c_out, c_in)
    return A


def svd_symbols(A: np.ndarray, compute_uv: bool = True):
    """Per-frequency SVD ``A_k = U_k S_k V_k^*`` (Sec. III "Convolution
    Theorem"; Algorithm 1 SVD step), with ``numpy.linalg.svd`` as the paper
    uses (Sec. IV "Runtime Analysis").

    ``A``: ``[..., c_out, c_in]`` complex.  Returns ``sigma [..., r]``
    (descending, ``r = min(c_out, c_in)``) and, if ``compute_uv``, the thin
    ``U [..., c_out, r]`` and ``V [..., c_in, r]`` with ``A = U diag(s) V^H``.
    """
    A = np.asarray(A, dtype=np.complex128)
    if not compute_uv:
        return np.linalg.svd(A, compute_uv=False)
    U, s, Vh = np.linalg.svd(A, full_matrices=False)
    V = np.conj(np.swapaxes(Vh, -1, -2))
    return s, U, V


def phase_normalize(U, V):
    """Fix the free phase of every singular pair (post-processing of
    Algorithm 1's SVD step; the paper leaves the phase open).  A pair
    ``(u_j, v_j)`` of ``A = U diag(s) V^H`` may be multiplied by any common
    ``e^{i phi}``; this picks the one that makes the entry of largest modulus
    of ``v_j`` real and positive, the lowest row on ties (of ``u_j`` when
    ``V`` is None).  ``U [..., c_out, r]`` and ``V [..., c_in, r]`` (either may
    be None); returns the normalised copies."""
    key = V if V is not None else U
    key = np.asarray(key, dtype=np.complex128)
    rows = key.shape[-2]
    out = []
    flat_key = key.reshape(-1, rows, key.shape[-1])
    phases = np.ones((flat_key.shape[0], key.shape[-1]), dtype=np.complex128)
    for b in range(flat_key.shape[0]):
        for j in range(key.shape[-1]):
            col = flat_key[b, :, j]
            mod2 = col.real ** 2 + col.imag ** 2
            i = int(np.argmax(mod2))          # first index of the maximum
            if mod2[i] > 0:
                phases[b, j] = np.conj(col[i]) / np.abs(col[i])
    phases = phases.reshape(key.shape[:-2] + (1, key.shape[-1]))
    for X in (U, V):
        out.append(None if X is None else np.asarray(X, dtype=np.complex128) * phases)
    return out[0], out[1]


def lfa_svd(W, n: int, m: int | None = None, compute_uv: bool = False, freqs=None):
    """Algorithm 1 end to end: symbols at every frequency, then their SVD."""
    A = symbols(W, n, m, freqs)
    return svd_symbols(A, compute_uv)


# ---------------------------------------------------------------------------
# The operator itself, unrolled (definition-level brute force)
# ---------------------------------------------------------------------------

def _unrolled(W, n: int, m: int, periodic: bool) -> np.ndarray:
    W = np.asarray(W, dtype=np.float64)
    c_out, c_in, kh, kw = W.shape
    y = tap_offsets(kh, kw)
    M = np.zeros((n * m * c_out, n * m * c_in), dtype=np.float64)
    for x1 in range(n):
        for x2 in range(m):
            row0 = (x1 * m + x2) * c_out
            for a in range(kh):
                for b in range(kw):
                    s1 = x1 + int(y[a, b, 0])
                    s2 = x2 + int(y[a, b, 1])
                    if periodic:
                        s1 %= n
                        s2 %= m
                    elif not (0 <= s1 < n and 0 <= s2 < m):
                        continue          # zero padding: f(x+y) = 0 off the grid
                    col0 = (s1 * m + s2) * c_in
                    M[row0:row0 + c_out, col0:col0 + c_in] += W[:, :, a, b]
    return M


def unrolled_operator(W, n: int, m: int | None = None) -> np.ndarray:
    """Dense matrix of ``(A*f)(x) = sum_y M_y f(x+y)`` with periodic boundary
    conditions (Sec. I matrix view; Sec. III "Convolutional Mappings").

    Vectors are indexed ``(x1*m + x2)*c + channel``.  Shape
    ``(n*m*c_out, n*m*c_in)``.  Taps that alias (kernel wider than the grid)
    add up, exactly as they do in the symbol.
    """
    m = n if m is None else m
    return _unrolled(W, n, m, periodic=True)


def dirichlet_operator(W, n: int, m: int | None = None) -> np.ndarray:
    """Same operator with zero padding, i.e. Dirichlet boundary conditions
    (Sec. III "Boundary Conditions"; Sec. IV, boundary-condition study)."""
    m = n if m is None else m
    return _unrolled(W, n, m, periodic=False)


# ---------------------------------------------------------------------------
# Strided convolutions: crystals with s*s points per unit cell
# ---------------------------------------------------------------------------

def strided_operator(W, n: int, m: int, s: int) -> np.ndarray:
    """Dense matrix of the stride-s periodic convolution
    ``y(x) = sum_y M_y f(s x + y)``: f on the n x m torus, y on the
    (n/s) x (m/s) torus (s divides n and m), taps centred as for stride 1.

    Rows ``(x1*(m/s) + x2)*c_out + o``, columns ``(z1*m + z2)*c_in + i``.
    Definition-level brute force (small grids only).
    """
    if n % s or m % s:
        raise ValueError("the stride must divide the grid")
    W = np.asarray(W, dtype=np.float64)
    c_out, c_in, kh, kw = W.shape
    y = tap_offsets(kh, kw)
    nc, mc = n // s, m // s
    M = np.zeros((nc * mc * c_out, n * m * c_in), dtype=np.float64)
    for x1 in range(nc):
        for x2 in range(mc):
            row0 = (x1 * mc + x2) * c_out
            for a in range(kh):
                for b in range(kw):
                    z1 = (s * x1 + int(y[a, b, 0])) % n
                    z2 = (s * x2 + int(y[a, b, 1])) % m
                    col0 = (z1 * m + z2) * c_in
                    M[row0:row0 + c_out, col0:col0 + c_in] += W[:, :, a, b]
    return M


def crystal_symbols(W, n: int, m: int, s: int) -> np.ndarray:
    """Symbols of the stride-s convolution, the input read as a crystal on the
    coarse lattice ``s Z^2`` with ``s*s*c_in`` points per unit cell and the
    output as the coarse torus with ``c_out`` points per cell (Sec. III
    "Introduction to Lattices and Crystals" and "Convolutional Mappings": a
    crystal torus has |det Z| times the points of its cell).

    The input point ``z = s X + d`` (cell X, position ``d = (d1, d2)`` in
    ``[0, s)^2``, channel i) is column ``i*s*s + d1*s + d2``; the Fourier mode
    of frequency k on the coarse torus ``T*_{n/s, m/s}`` takes the value
    ``e^{2 pi i <k, X>}`` there (the cell's coordinates; adding the point's
    offset ``d/s`` inside the cell multiplies each column by a unit phase,
    which leaves sigma and U unchanged).  A tap at offset y reaches the point
    ``d = y mod s`` of cell ``X + floor(y / s)``, so

        A_k[o, i*s*s + d1*s + d2] = sum over taps y with y mod s = d of
                                    M_y[o, i] e^{2 pi i <k, floor(y/s)>}.

    Returns ``[n/s, m/s, c_out, s*s*c_in]`` complex128.
    """
    if n % s or m % s:
        raise ValueError("the stride must divide the grid")
    W = np.asarray(W, dtype=np.float64)
    c_out, c_in, kh, kw = W.shape
    y = tap_offsets(kh, kw)
    nc, mc = n // s, m // s
    A = np.zeros((nc, mc, c_out, c_in * s * s), dtype=np.complex128)
    p = np.arange(nc)[:, None]
    q = np.arange(mc)[None, :]
    for a in range(kh):
        for b in range(kw):
            Y1, d1 = divmod(int(y[a, b, 0]), s)      # floor division, d in [0, s)
            Y2, d2 = divmod(int(y[a, b, 1]), s)
            ph = np.exp(2j * np.pi * (np.mod(p * Y1, nc) / nc + np.mod(q * Y2, mc) / mc))
            cols = np.arange(c_in) * s * s + d1 * s + d2
            A[:, :, :, cols] += ph[:, :, None, None] * W[None, None, :, :, a, b]
    return A


# ---------------------------------------------------------------------------
# Global singular vectors (lift)
# ---------------------------------------------------------------------------

def fourier_basis(n: int, m: int, p: int, q: int, c: int) -> np.ndarray:
    """Orthonormal Fourier modes of one frequency on the crystal torus with c
    collocated channels (Sec. III "Convolution Theorem"): column ``i`` is
    ``e^{2 pi i <k, x>} e_i / sqrt(n m)``.  Shape ``(n*m*c, c)``."""
    k = frequency_grid(n, m)[p, q]
    x1, x2 = np.meshgrid(np.arange(n), np.arange(m), indexing="ij")
    wave = np.exp(2j * np.pi * (k[0] * x1 + k[1] * x2)).ravel() / np.sqrt(n * m)
    F = np.zeros((n * m * c, c), dtype=np.complex128)
    for i in range(c):
        F[i::c, i] = wave
    return F


def lift(U, V, n: int, m: int, p: int, q: int):
    """Global singular vectors ``U_hat = F^out_k U_k`` and ``V_hat = F^in_k V_k``
    (Sec. III "Convolution Theorem")."""
    Fo = fourier_basis(n, m, p, q, U.shape[0])
    Fi = fourier_basis(n, m, p, q, V.shape[0])
    return Fo @ U, Fi @ V


# ---------------------------------------------------------------------------
# Spectral functions of the operator applied through the per-symbol SVD
# ---------------------------------------------------------------------------

def spectral_factor(sigma, kind: str, param: float = 0.0):
    """``f(sigma)`` of the spectral functions applied below: ``identity`` (the
    operator itself), ``clip`` (``min(sigma, param)``: the operator with its
    singular values clipped at ``param``), ``truncate`` (``sigma`` above
    ``param``, else 0: the low-rank truncation of the operator) and ``pinv``
    (``1/sigma`` above the absolute cut-off ``param``, else 0: the
    pseudo-inverse restricted to the kept singular values)."""
    s = np.asarray(sigma, dtype=np.float64)
    if kind == "identity":
        return s.copy()
    if kind == "pinv":
        out = np.zeros_like(s)
        keep = s > param
        out[keep] = 1.0 / s[keep]
        return out
    if kind == "clip":
        return np.minimum(s, param)
    if kind == "truncate":
        return np.where(s > param, s, 0.0)
    raise ValueError(kind)


def apply_spectral(W, x, n: int, m: int | None, kind: str, param: float = 0.0):
    """A spectral function of the periodic operator ``A = U Sigma V^*``
    applied to ``x``, evaluated frequency by frequency (Sec. III "Convolution
    Theorem": the global singular vectors are Fourier modes times the
    singular vectors of the symbols):

    * ``identity``, ``clip`` and ``truncate``: ``y = U f(Sigma) V^* x``, ``x [B, c_in, n, m]``
      real, ``y [B, c_out, n, m]``;
    * ``pinv``: ``y = V f(Sigma) U^* x`` (the pseudo-inverse maps back from the
      output channels), ``x [B, c_out, n, m]``, ``y [B, c_in, n, m]``.

    With ``x_hat_k = sum_x x(x) e^{-2 pi i <k, x>}`` the operator maps
    ``x_hat_k`` to ``A_k x_hat_k``; here each ``x_hat_k`` goes to
    ``U_k f(S_k) V_k^* x_hat_k`` (or ``V_k f(S_k) U_k^* x_hat_k``) and ``y`` is
    the inverse transform (``1/(n m)`` and ``e^{+2 pi i <k, x>}``).  Returns
    the real part in float64 (the imaginary part vanishes for real W and x).
    """
    m = n if m is None else m
    x = np.asarray(x, dtype=np.float64)
    xh = np.fft.fft2(x, axes=(-2, -1))
    S, U, V = svd_symbols(symbols(W, n, m), compute_uv=True)  # [n, m, ...]
    f = spectral_factor(S, kind, param)                      # [n, m, r]
    left, right = (V, U) if kind == "pinv" else (U, V)
    z = np.einsum("pqir,bipq->bpqr", np.conj(right), xh)
    yh = np.einsum("pqor,pqr,bpqr->bopq", left, f, z)
    return np.real(np.fft.ifft2(yh, axes=(-2, -1)))


def apply_spectral_dense(W, x, n: int, m: int | None, kind: str, param: float = 0.0):
    """The same spectral function from the SVD of the dense unrolled operator
    (definition-level brute force, small grids only)."""
    m = n if m is None else m
    x = np.asarray(x, dtype=np.float64)
    B, c = x.shape[:2]
    A = unrolled_operator(W, n, m)
    Ud, Sd, Vdh = np.linalg.svd(A)
    r = Sd.size
    f = spectral_factor(Sd, kind, param)
    if kind == "pinv":
        left, right = Vdh[:r].conj().T, Ud[:, :r]
    else:
        left, right = Ud[:, :r], Vdh[:r].conj().T
    xv = np.transpose(x, (0, 2, 3, 1)).reshape(B, n * m * c)   # (x1 m + x2) c + channel
    yv = ((xv @ right.conj()) * f) @ left.T
    c_y = left.shape[0] // (n * m)
    return np.transpose(yv.reshape(B, n, m, c_y), (0, 3, 1, 2))


# ---------------------------------------------------------------------------
# Top-k and gradient of a sum of singular values
# ---------------------------------------------------------------------------

def topk(sigma: np.ndarray, k: int):
    """The k largest singular values of one layer, ``sigma [n, m, r]``.

    Order: value descending, ties by flat index ``(p, q, j)`` ascending.
    Returns ``(vals [k], idx [k, 3])`` with idx rows ``(p, q, j)``.
    """
    s = np.asarray(sigma, dtype=np.float64)
    n, m, r = s.shape
    flat = s.ravel()
    order = np.lexsort((np.arange(flat.size), -flat))[:k]
    p, rem = np.divmod(order, m * r)
    q, j = np.divmod(rem, r)
    return flat[order], np.stack([p, q, j], axis=1)


def sigma_grad(W, n: int, m: int | None, picks, grad_out=None):
    """Gradient of ``L = sum_s g_s * sigma_{j_s}(k_s)`` with respect to W.

    For a simple singular value, ``d sigma = Re(u^H dA v)``; with
    ``dA/dW[o,i,a,b] = e^{2 pi i <k, y_ab>} E_oi`` this gives
    ``dsigma/dW[o,i,a,b] = Re(e^{-2 pi i <k, y_ab>} u[o] conj(v[i]))``.

    ``picks``: ``(S, 3)`` integer ``(p, q, j)``; ``grad_out``: ``(S,)`` weights
    (default ones).  Singular vectors come from ``numpy.linalg.svd`` of the
    oracle's own symbols.  Returns float64 ``[c_out, c_in, kh, kw]``.
    """
    m = n if m is None else m
    W = np.asarray(W, dtype=np.float64)
    c_out, c_in, kh, kw = W.shape
    picks = np.asarray(picks, dtype=np.int64).reshape(-1, 3)
    g = np.ones(len(picks)) if grad_out is None else np.asarray(grad_out, np.float64)
    dW = np.zeros_like(W)
    freqs = picks[:, :2]
    A = symbols(W, n, m, freqs)
    ph = phase_factors(n, m, kh, kw, freqs)
    for s in range(len(picks)):
        _, U, V = svd_symbols(A[s], compute_uv=True)
        j = int(picks[s, 2])
        outer = np.outer(U[:, j], np.conj(V[:, j]))        # u v^H, c_out x c_in
        dW += g[s] * np.real(np.conj(ph[s])[None, None, :, :] * outer[:, :, None, None])
    return dW


# ---------------------------------------------------------------------------
# Error metric
# ---------------------------------------------------------------------------

def sigma_error(sig_test, sig_ref):
    """Normwise per-symbol singular-value error
    ``max_{k, j} |s_test - s_ref| / max_j s_ref(k)`` (zero symbols count as
    absolute error)."""
    st = np.asarray(sig_test, dtype=np.float64)
    sr = np.asarray(sig_ref, dtype=np.float64)
    smax = sr.max(axis=-1, keepdims=True)
    smax = np.where(smax > 0, smax, 1.0)
    return float(np.max(np.abs(st - sr) / smax))
