"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every expected value is computed here, on the CPU, by ``oracle`` from the
same seeded weights the GPU receives (float32 weights are upcast, so errors
measure the computation, not the input rounding).
"""

import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import (banner, check_projectors, check_vectors, grad_errors, sigma_gate, to_np)

pytestmark = pytest.mark.gpu

DEV = "cuda"


def lfa():
    import paper_2506_05617_amd as m
    return m


def _w(W):
    return torch.from_numpy(np.ascontiguousarray(W)).to(DEV)


def _grad_check(W64, l, picks, g, dW, tag, ref=None):
    """dW of L = sum_s g_s sigma_s against the oracle's gradient for the same
    picks, elementwise for separated picks (gpu_util.grad_errors)."""
    picks = np.asarray(picks)
    if ref is None:
        ref = oracle.sigma_grad(W64, l.n, l.m, picks, g)
    S_sym = oracle.lfa_svd(W64, l.n, l.m, freqs=picks[:, :2])
    return grad_errors(to_np(dW), ref, S_sym, picks, g, tag)


# ---------------------------------------------------------------- symbols --

SYMBOL_CASES = [
    # c_out, c_in, kh, kw, n, m, dtype
    (16, 16, 3, 3, 32, 32, np.float64),
    (16, 16, 3, 3, 32, 32, np.float32),
    (64, 64, 3, 3, 9, 7, np.float32),        # non-square grid, ragged tiles
    (5, 3, 3, 3, 6, 5, np.float32),
    (3, 64, 3, 3, 8, 8, np.float32),         # c_out < c_in
    (64, 64, 7, 7, 11, 11, np.float32),      # 7x7 kernel
    (7, 9, 1, 1, 3, 4, np.float64),          # 1x1 kernel
    (2, 2, 2, 4, 5, 6, np.float32),          # even kernel extents
]


@pytest.mark.parametrize("case", SYMBOL_CASES)
def test_symbols_match_oracle(case):
    c_out, c_in, kh, kw, n, m, dt = case
    banner(f"symbols {case}")
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=3, dtype=dt)
    A = to_np(lfa().symbols(_w(W), n, m))
    ref = oracle.symbols(W.astype(np.float64), n, m)
    scale = np.max(np.sum(np.abs(W.astype(np.float64)), axis=(2, 3)))
    eps = 2.0 ** -24 if dt == np.float32 else 2.0 ** -53
    err = np.max(np.abs(A - ref))
    # each element sums kh*kw products of a weight and a phase rounded once
    assert err <= 4 * (kh * kw + 2) * eps * scale, err


@pytest.mark.parametrize("asm,gate", [("mfma", 1e-6), ("bf16x3", 1e-6), ("bf16x2", 3e-5)])
@pytest.mark.parametrize("shape", [(64, 64, 3, 3, 9, 7), (64, 64, 7, 7, 10, 10), (5, 3, 3, 3, 4, 6),
                                   (2, 2, 2, 4, 5, 6),       # even kernel extents
                                   (4, 3, 1, 9, 3, 10),      # one kernel row
                                   (3, 2, 17, 3, 18, 4)])    # 17 rows: the direct contraction
def test_symbols_matrix_cores(asm, gate, shape):
    c_out, c_in, kh, kw, n, m = shape
    banner(f"symbols {asm} {shape}")
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=5, dtype=np.float32)
    A = to_np(lfa().symbols(_w(W), n, m, asm=asm))
    ref = oracle.symbols(W.astype(np.float64), n, m)
    scale = np.max(np.sum(np.abs(W.astype(np.float64)), axis=(2, 3)))
    err = np.max(np.abs(A - ref)) / scale
    assert err <= gate, err


# -------------------------------------------------------------------- SVD --

SVD_CASES = [
    # c_out, c_in, kh, kw, n, m, dtype, vectors
    (16, 16, 3, 3, 32, 32, np.float64, True),      # the 16-channel 32x32 layer, FP64 mode
    (16, 16, 3, 3, 32, 32, np.float32, True),
    (4, 4, 3, 3, 8, 8, np.float64, False),
    (5, 3, 3, 3, 6, 5, np.float32, True),          # odd column count
    (3, 5, 3, 3, 5, 6, np.float32, True),          # c_out < c_in
    (1, 1, 3, 3, 7, 7, np.float32, True),
    (64, 3, 3, 3, 8, 8, np.float32, True),         # first ResNet layer shape
    (64, 64, 3, 3, 6, 5, np.float32, True),
    (64, 64, 3, 3, 6, 5, np.float64, True),
    (128, 64, 3, 3, 4, 4, np.float32, True),
    (128, 128, 3, 3, 3, 3, np.float32, True),      # vectors exceed LDS: global storage
    (128, 128, 3, 3, 3, 3, np.float32, False),
    (256, 128, 3, 3, 3, 3, np.float32, True),
    (64, 64, 7, 7, 7, 7, np.float32, False),
    (512, 256, 3, 3, 3, 3, np.float32, True),      # rectangular 512x256 symbols
]


def _run_svd(W, n, m, vectors):
    out = lfa().svd(_w(W), n, m, compute_uv=vectors, return_info=True)
    (S, U, V), info = (out[0], out[1]) if vectors else ((out[0], None, None), out[1])
    torch.cuda.synchronize()
    return S, U, V, to_np(info)


@pytest.mark.parametrize("case", SVD_CASES)
def test_svd_matches_oracle(case):
    c_out, c_in, kh, kw, n, m, dt, vectors = case
    banner(f"svd {case}")
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=11, dtype=dt)
    S, U, V, info = _run_svd(W, n, m, vectors)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    A = oracle.symbols(W.astype(np.float64), n, m)
    S_ref, U_ref, V_ref = oracle.svd_symbols(A, compute_uv=True)
    e = oracle.sigma_error(to_np(S), S_ref)
    assert e <= sigma_gate(tdt), f"sigma error {e:.3e}"
    assert np.all(np.diff(to_np(S), axis=-1) <= 0), "not sorted"
    assert info[0] == 0 and info[3] == 0, f"info {info}"
    if vectors:
        check_vectors(A, to_np(S), to_np(U), to_np(V), tdt, str(case))
        check_projectors(S_ref, U_ref, V_ref, to_np(U), to_np(V), tdt, str(case))


# (c_out, c_in, kh, kw, n, m, asm, vectors)
MAT_CASES = [
    (8, 6, 5, 5, 7, 10, None, True),        # 25 taps: matrix-core assembly by default; odd n
    (6, 8, 5, 5, 10, 7, None, False),       # odd m, c_out < c_in
    (5, 3, 3, 3, 4, 6, "mfma", True),
    (12, 12, 9, 9, 9, 10, "bf16x3", False),  # 81 taps: the kernel without held phases
    (16, 16, 3, 3, 9, 9, "bf16x2", True),
]


@pytest.mark.parametrize("case", MAT_CASES)
def test_materialised_assembly_svd_matches_oracle(case):
    """The SVD with the symbols assembled on matrix cores first (only the
    canonical symbol of each conjugate pair is formed): sigma over the whole
    grid against the oracle, and with vectors the residuals of every symbol,
    mirrors included."""
    c_out, c_in, kh, kw, n, m, asm, vectors = case
    banner(f"materialised svd {case}")
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=12, dtype=np.float32)
    out, info = lfa().svd(_w(W), n, m, asm=asm, compute_uv=vectors, return_info=True)
    torch.cuda.synchronize()
    S = out[0] if vectors else out
    info = to_np(info)
    assert info[0] == 0 and info[3] == 0, f"info {info}"
    A = oracle.symbols(W.astype(np.float64), n, m)
    S_ref = oracle.svd_symbols(A, compute_uv=False)
    gate = 3e-5 if asm == "bf16x2" else sigma_gate(torch.float32)
    e = oracle.sigma_error(to_np(S), S_ref)
    assert e <= gate, f"sigma error {e:.3e}"
    if vectors and asm != "bf16x2":
        check_vectors(A, to_np(S), to_np(out[1]), to_np(out[2]), torch.float32, str(case))


# (c_out, c_in, kh, kw, n, m, dtype)
PHASE_CASES = [
    (16, 12, 3, 3, 5, 6, np.float64),      # register kernel, FP64
    (24, 40, 3, 3, 4, 5, np.float32),      # wide layer: G = A^H
    (64, 64, 3, 3, 6, 5, np.float32),      # the headline's symbols (work queue)
    (160, 96, 3, 3, 3, 4, np.float32),     # blocked kernel
    (256, 128, 3, 3, 4, 4, np.float32),    # QR preconditioning (tall)
]


@pytest.mark.parametrize("case", PHASE_CASES)
def test_phase_normalize_matches_oracle(case, monkeypatch):
    """LFA_PHASE_NORMALIZE: sigma bitwise that of the plan without the flag,
    each (u_j, v_j) that plan's pair times one common phase, the
    largest-modulus entry of every v_j real and positive, and, for simple
    singular values whose v_j has a clear largest entry, U and V elementwise
    equal to the oracle's SVD after the oracle's phase_normalize."""
    c_out, c_in, kh, kw, n, m, dt = case
    if c_out >= 256:
        monkeypatch.setenv("LFA_QR", "1")
    banner(f"phase normalize {case}")
    _, W = workloads.random_layer(c_out, c_in, kh, kw, n, m, seed=13, dtype=dt)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    S0, U0, V0 = lfa().svd(_w(W), n, m, compute_uv=True)
    (S, U, V), info = lfa().svd(_w(W), n, m, compute_uv=True, phase_normalize=True, return_info=True)
    torch.cuda.synchronize()
    assert to_np(info)[0] == 0
    assert torch.equal(S, S0)
    S, U, V, U0, V0 = to_np(S), to_np(U), to_np(V), to_np(U0), to_np(V0)
    # one common phase per pair: v_j = v0_j z_j and u_j = u0_j z_j, |z_j| = 1
    z = np.sum(np.conj(V0) * V, axis=-2)                      # [n, m, r]
    np.testing.assert_allclose(np.abs(z), 1, atol=1e-5 if dt == np.float32 else 1e-12)
    np.testing.assert_allclose(V, V0 * z[..., None, :], atol=1e-6 if dt == np.float32 else 1e-13)
    np.testing.assert_allclose(U, U0 * z[..., None, :], atol=1e-6 if dt == np.float32 else 1e-13)
    # an entry of modulus max |v_j| is exactly real and positive
    mod = np.abs(V)
    top = mod.max(axis=-2, keepdims=True)
    realpos = (V.imag == 0) & (V.real > 0) & (mod >= top * (1 - 1e-6))
    assert np.all(realpos.any(axis=-2))
    # the oracle's normalised SVD, where the pair and its phase are unique
    A = oracle.symbols(W.astype(np.float64), n, m)
    S_ref, U_ref, V_ref = oracle.svd_symbols(A)
    U_ref, V_ref = oracle.phase_normalize(U_ref, V_ref)
    eps = 1e-6 if dt == np.float32 else 1e-13
    smax = S_ref[..., :1]
    d = np.abs(np.diff(S_ref, axis=-1))
    gap = np.full(S_ref.shape, np.inf)
    gap[..., :-1] = np.minimum(gap[..., :-1], d)
    gap[..., 1:] = np.minimum(gap[..., 1:], d)
    rel_gap = gap / smax
    mref = np.sort(np.abs(V_ref), axis=-2)
    sep = (mref[..., -1, :] - mref[..., -2, :]) / mref[..., -1, :]
    ok = (rel_gap > 1e-3) & (sep > 1e-3) & (S_ref > 1e-3 * smax)
    assert ok.sum() > 0
    bound = eps * (10 + 1 / rel_gap) * (1 + 1 / sep)
    ev = np.max(np.abs(V - V_ref), axis=-2)
    eu = np.max(np.abs(U - U_ref), axis=-2)
    assert np.all(ev[ok] <= bound[ok]), f"V: worst {np.max(ev[ok] / bound[ok]):.3e} of the bound"
    assert np.all(eu[ok] <= bound[ok]), f"U: worst {np.max(eu[ok] / bound[ok]):.3e} of the bound"


def test_phase_normalize_u_alone():
    """LFA_PHASE_NORMALIZE with U alone: the rule applies to u_j, and the
    pairs are those of the plan without the flag times one phase each."""
    banner("phase normalize, U alone")
    _, W = workloads.random_layer(32, 24, 3, 3, 4, 6, seed=14, dtype=np.float32)
    spec = lfa().LayerSpec(32, 24, 3, 3, 4, 6)
    S0, U0, _, _ = lfa().Plan([spec], torch.float32, True, False).svd([_w(W)])
    S1, U1, V1, _ = lfa().Plan([spec], torch.float32, True, False, phase_normalize=True).svd([_w(W)])
    torch.cuda.synchronize()
    assert V1[0] is None
    assert torch.equal(S0[0], S1[0])
    U0, U1 = to_np(U0[0]), to_np(U1[0])
    z = np.sum(np.conj(U0) * U1, axis=-2)
    np.testing.assert_allclose(np.abs(z), 1, atol=1e-5)
    np.testing.assert_allclose(U1, U0 * z[..., None, :], atol=1e-6)
    mod = np.abs(U1)
    realpos = (U1.imag == 0) & (U1.real > 0) & (mod >= mod.max(axis=-2, keepdims=True) * (1 - 1e-6))
    assert np.all(realpos.any(axis=-2))


def test_brute_force_size_against_dense_operator():
    """4->4 channels on the 8x8 grid: sigma of the GPU path == sigma of the
    dense 256x256 operator (LAPACK on the CPU)."""
    banner("brute force n=8 c=4")
    L, W = workloads.brute_force_small()
    S = to_np(lfa().svd(_w(W), L.n, L.m))
    dense = oracle.unrolled_operator(W, L.n, L.m)
    s_dense = np.sort(np.linalg.svd(dense, compute_uv=False))[::-1]
    np.testing.assert_allclose(np.sort(S.ravel())[::-1], s_dense, rtol=0, atol=1e-12 * s_dense[0])


def test_identity_and_zero_kernels():
    banner("identity / zero kernels")
    c = 24
    W = np.zeros((c, c, 3, 3), np.float32)
    W[:, :, 1, 1] = np.eye(c)
    S, U, V = lfa().svd(_w(W), 5, 5, compute_uv=True)
    np.testing.assert_allclose(to_np(S), 1.0, atol=1e-6)
    # all-zero weights: sigma = 0, U must still be orthonormal (completion)
    Z = np.zeros((12, 7, 3, 3), np.float32)
    S, U, V = lfa().svd(_w(Z), 4, 3, compute_uv=True)
    assert np.all(to_np(S) == 0)
    Ud, Vd = to_np(U).astype(np.complex128), to_np(V).astype(np.complex128)
    eye = np.eye(7)
    assert np.max(np.abs(np.conj(np.swapaxes(Ud, -1, -2)) @ Ud - eye)) < 1e-6
    assert np.max(np.abs(np.conj(np.swapaxes(Vd, -1, -2)) @ Vd - eye)) < 1e-6


@pytest.mark.parametrize("shape", [(64, 32, 4), (512, 256, 3)])
def test_rank_one_taps(shape):
    """Exactly rank-one taps: rank A_k <= 9, the other singular values vanish;
    sum sigma^2 = n^2 ||W||_F^2; left vectors of zero sigma stay orthonormal."""
    c_out, c_in, n = shape
    banner(f"rank-one taps {shape}")
    L, W = workloads.rank_one_taps(c_out=c_out, c_in=c_in, n=n)
    S, U, V = lfa().svd(_w(W), n, n, compute_uv=True)
    S, U, V = to_np(S), to_np(U), to_np(V)
    smax = S[..., :1]
    assert np.all(S[..., 9:] <= 1e-5 * smax)
    W64 = W.astype(np.float64)
    parseval = np.sum(S.astype(np.float64) ** 2) / (n * n * np.sum(W64 ** 2))
    assert abs(parseval - 1) <= 1e-6, parseval
    A = oracle.symbols(W64, n, n)
    S_ref = oracle.svd_symbols(A, compute_uv=False)
    assert oracle.sigma_error(S, S_ref) <= 1e-5
    check_vectors(A, S, U, V, torch.float32, "rank-one")


# ------------------------------------------------------- full-size sample --

def test_single_layer_64_full_size_sampled():
    """64->64 channels on the 64x64 grid, sigma + U + V, at full size in the
    launch configuration the benchmark times; 48 sampled symbols checked
    against the oracle one by one, Parseval over the whole grid."""
    banner("64x64 layer full size")
    L, W = workloads.single_layer_64()
    S, U, V = lfa().svd(_w(W), L.n, L.m, compute_uv=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    fr = rng.integers(0, L.n, size=(48, 2))
    fr[0] = (0, 0)
    fr[1] = (L.n - 1, L.m - 1)
    A = oracle.symbols(W.astype(np.float64), L.n, L.m, fr)
    S_ref, U_ref, V_ref = oracle.svd_symbols(A, compute_uv=True)
    Sg = to_np(S)[fr[:, 0], fr[:, 1]]
    Ug = to_np(U)[fr[:, 0], fr[:, 1]]
    Vg = to_np(V)[fr[:, 0], fr[:, 1]]
    assert oracle.sigma_error(Sg, S_ref) <= 1e-5
    check_vectors(A, Sg, Ug, Vg, torch.float32, "64x64")
    check_projectors(S_ref, U_ref, V_ref, Ug, Vg, torch.float32, "64x64")
    W64 = W.astype(np.float64)
    ps = np.sum(to_np(S).astype(np.float64) ** 2) / (L.n * L.m * np.sum(W64 ** 2))
    assert abs(ps - 1) <= 1e-6


# ------------------------------------------- repeated vectors, 64 x 64 --

@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_register_kernel_vectors_repeated(dt):
    """The register kernel's two waves (working matrix and accumulator) share
    LDS state; a missing synchronisation shows up as a wrong V on some runs
    only.  Several seeds, every symbol checked (residual and orthonormality)."""
    banner(f"repeated 64x64 vectors {dt.__name__}")
    tdt = torch.float32 if dt == np.float32 else torch.float64
    for seed in (11, 12, 13, 14):
        _, W = workloads.random_layer(64, 64, 3, 3, 6, 5, seed=seed, dtype=dt)
        S, U, V, info = _run_svd(W, 6, 5, True)
        A = oracle.symbols(W.astype(np.float64), 6, 5)
        check_vectors(A, to_np(S), to_np(U), to_np(V), tdt, f"seed {seed}")


# ------------------------------------------------------------ work queue --

def _plan_svd(W, n, m, vectors, queue):
    """SVD of one layer by a fresh plan created with LFA_WAVE_QUEUE = queue
    (None: automatic)."""
    import os
    c_out, c_in, kh, kw = W.shape
    old = os.environ.pop("LFA_WAVE_QUEUE", None)
    try:
        if queue is not None:
            os.environ["LFA_WAVE_QUEUE"] = str(queue)
        plan = lfa().Plan([lfa().LayerSpec(c_out, c_in, kh, kw, n, m)],
                          torch.float32 if W.dtype == np.float32 else torch.float64, vectors, vectors)
    finally:
        os.environ.pop("LFA_WAVE_QUEUE", None)
        if old is not None:
            os.environ["LFA_WAVE_QUEUE"] = old
    S, U, V, info = plan.svd([_w(W)])
    torch.cuda.synchronize()
    return plan, S[0], (U[0] if vectors else None), (V[0] if vectors else None), to_np(info[0])


QUEUE_CASES = [
    # c_out, c_in, n, m, dtype, vectors, LFA_WAVE_QUEUE of the queued run
    (16, 16, 24, 20, np.float32, True, 1),    # four symbols per wave
    (16, 16, 24, 20, np.float64, True, 2),
    (40, 24, 10, 9, np.float32, True, 3),     # 64 rows, 32 padded columns
    (24, 40, 9, 10, np.float64, False, 1),    # c_out < c_in, sigma only
    (5, 3, 6, 5, np.float32, True, 1),        # smallest shape (4 columns)
    (64, 64, 7, 6, np.float32, False, 2),
]


@pytest.mark.parametrize("case", QUEUE_CASES)
def test_work_queue_is_bitwise_the_plain_launch(case):
    """The work-queue launch (groups run a few sweeps per turn, their state
    saved and restored in between) performs the same arithmetic as one
    uninterrupted run: sigma, U, V and the sweep counts are bitwise equal."""
    c_out, c_in, n, m, dt, vectors, k = case
    banner(f"work queue {case}")
    _, W = workloads.random_layer(c_out, c_in, 3, 3, n, m, seed=21, dtype=dt)
    pq, Sq, Uq, Vq, iq = _plan_svd(W, n, m, vectors, k)
    assert pq.queue_info(0)[1] == k
    pp, Sp, Up, Vp, ip = _plan_svd(W, n, m, vectors, 0)
    assert pp.queue_info(0)[1] == 0
    assert np.array_equal(iq, ip), (iq, ip)
    assert torch.equal(Sq, Sp)
    if vectors:
        assert torch.equal(Uq, Up) and torch.equal(Vq, Vp)
    S_ref = oracle.lfa_svd(W.astype(np.float64), n, m)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    assert oracle.sigma_error(to_np(Sq), S_ref) <= sigma_gate(tdt)


@pytest.mark.parametrize("vectors", [True, False])
def test_work_queue_headline_shape(vectors):
    """64 -> 64 channels on the 64 x 64 grid: 2050 groups, more than the
    device holds at once, so the automatic choice is the work queue.  Bitwise
    equal to the plain launch, every symbol checked against the oracle, and
    repeated (the queue state is rebuilt by every call)."""
    banner(f"work queue headline vectors={vectors}")
    L, W = workloads.single_layer_64()
    pq, Sq, Uq, Vq, iq = _plan_svd(W, 64, 64, vectors, None)
    resident, seg = pq.queue_info(0)
    assert 0 < resident < 2050 and seg >= 1, (resident, seg)
    _, Sp, Up, Vp, ip = _plan_svd(W, 64, 64, vectors, 0)
    assert np.array_equal(iq, ip) and iq[0] == 0 and iq[3] == 0, (iq, ip)
    assert torch.equal(Sq, Sp)
    if vectors:
        assert torch.equal(Uq, Up) and torch.equal(Vq, Vp)
    for _ in range(2):
        S2, U2, V2, i2 = pq.svd([_w(W)])
        torch.cuda.synchronize()
        assert torch.equal(S2[0], Sq) and np.array_equal(to_np(i2[0]), iq)
        if vectors:
            assert torch.equal(U2[0], Uq) and torch.equal(V2[0], Vq)
    S_ref = oracle.lfa_svd(W.astype(np.float64), 64, 64)
    assert oracle.sigma_error(to_np(Sq), S_ref) <= sigma_gate(torch.float32)


def test_work_queue_caller_symbols():
    """lfa_svd_symbols (symbols handed in by the caller: every frequency is
    decomposed, no conjugate pairing) through the forced work queue, bitwise
    equal to the plain launch and within the sigma gate of the oracle."""
    import os
    banner("work queue, caller symbols")
    n, m = 10, 9
    _, W = workloads.random_layer(40, 24, 3, 3, n, m, seed=23, dtype=np.float32)
    A = lfa().symbols(_w(W), n, m)
    res = []
    for q in ("2", "0"):
        old = os.environ.pop("LFA_WAVE_QUEUE", None)
        os.environ["LFA_WAVE_QUEUE"] = q
        try:
            plan = lfa().Plan([lfa().LayerSpec(40, 24, 3, 3, n, m)], torch.float32, True, True)
        finally:
            os.environ.pop("LFA_WAVE_QUEUE", None)
            if old is not None:
                os.environ["LFA_WAVE_QUEUE"] = old
        assert plan.queue_info(0)[1] == int(q)
        S, U, V, info = plan.svd_symbols([A])
        torch.cuda.synchronize()
        res.append((S[0], U[0], V[0], to_np(info[0])))
    (Sq, Uq, Vq, iq), (Sp, Up, Vp, ip) = res
    assert np.array_equal(iq, ip) and iq[0] == 0 and iq[3] == 0, (iq, ip)
    assert torch.equal(Sq, Sp) and torch.equal(Uq, Up) and torch.equal(Vq, Vp)
    S_ref = oracle.svd_symbols(to_np(A).astype(np.complex128), compute_uv=False)
    assert oracle.sigma_error(to_np(Sq), S_ref) <= sigma_gate(torch.float32)


# ------------------------------------------------------ paper-scale grid --

def test_paper_scale_n16384_sampled():
    """The runtime study's largest case (Sec. IV, Table II): 16 -> 16 channels,
    3x3, 16384 x 16384 grid, sigma only (4.29e9 values, 17 GB).  64 sampled
    symbols against the oracle, including k = 0, the last frequency and the
    real symbol at (n/2, n/2); Parseval over the whole grid."""
    banner("paper scale n=16384")
    n = 16384
    L, W = workloads.paper_scale(n)
    S, info = lfa().svd(_w(W), n, n, compute_uv=False, return_info=True)
    torch.cuda.synchronize()
    assert info[0] == 0 and info[3] == 0, f"info {info}"
    rng = np.random.default_rng(3)
    fr = rng.integers(0, n, size=(64, 2))
    fr[0] = (0, 0)
    fr[1] = (n - 1, n - 1)
    fr[2] = (n // 2, n // 2)
    fr[3] = (n // 2, 0)
    Sg = S[fr[:, 0], fr[:, 1]].cpu().numpy()
    S_ref = oracle.lfa_svd(W.astype(np.float64), n, n, freqs=fr)
    assert oracle.sigma_error(Sg, S_ref) <= 1e-5
    ss = torch.sum(S.double() ** 2).item()
    assert abs(ss / (n * n * np.sum(W.astype(np.float64) ** 2)) - 1) <= 1e-5
    del S
    torch.cuda.empty_cache()


# --------------------------------------------- persistent, top-k, gradient --

def _small_stack(seed=4):
    shapes = ((3, 64, 8), (64, 64, 8), (64, 128, 4), (128, 128, 4), (128, 256, 2), (256, 256, 2),
              (256, 512, 1), (512, 512, 1))
    # n=1 grids need a 1x1 kernel; keep 3x3 and n >= 3 instead
    shapes = tuple((ci, co, max(n, 3)) for ci, co, n in shapes)
    return workloads.resnet18_stack(seed=seed, shapes=shapes)


def test_persistent_matches_plain():
    banner("persistent vs plain")
    layers, Ws = _small_stack()
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs)
    Wt = [_w(W) for W in Ws]
    S1, _, _, i1 = plan.svd(Wt, persistent=False)
    S2, _, _, i2 = plan.svd(Wt, persistent=True)
    torch.cuda.synchronize()
    for l, W, a, b in zip(layers, Ws, S1, S2):
        S_ref = oracle.lfa_svd(W.astype(np.float64), l.n, l.m)
        assert oracle.sigma_error(to_np(a), S_ref) <= 1e-5
        assert oracle.sigma_error(to_np(b), S_ref) <= 1e-5
    assert int(to_np(i2)[:, 0].sum()) == 0


def test_topk_matches_oracle():
    banner("topk")
    layers, Ws = _small_stack(seed=7)
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs)
    S, _, _, _ = plan.svd([_w(W) for W in Ws])
    k = 8
    vals, idx = plan.topk(S, k)
    vals, idx = to_np(vals), to_np(idx)
    for li, (l, s) in enumerate(zip(layers, S)):
        s = to_np(s)
        ref_vals, _ = oracle.topk(s, k)                   # same values, same order rule
        np.testing.assert_array_equal(vals[li], ref_vals.astype(s.dtype))
        p, q, j = idx[li].T
        np.testing.assert_array_equal(s[p, q, j], vals[li])
        # against the FP64 oracle's spectrum: the k largest values agree
        S_ref = oracle.lfa_svd(Ws[li].astype(np.float64), l.n, l.m)
        ov, _ = oracle.topk(S_ref, k)
        np.testing.assert_allclose(vals[li], ov, rtol=0, atol=1e-5 * ov[0])


def test_sigma_grad_matches_oracle_and_adjoint():
    banner("sigma grad")
    layers, Ws = _small_stack(seed=9)
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    k = 8
    plan = lfa().Plan(specs)
    Wt = [_w(W) for W in Ws]
    S, _, _, _ = plan.svd(Wt)
    vals, idx = plan.topk(S, k)
    g = torch.linspace(0.5, 1.5, k, device=DEV).repeat(len(layers), 1)
    dW = plan.sigma_grad(Wt, idx, g)
    dWp = plan.sigma_grad(Wt, idx, g, persistent=True)
    # the same adjoint from full U, V of a vectors plan
    plan_uv = lfa().Plan(specs, want_u=True, want_v=True)
    _, U, V, _ = plan_uv.svd(Wt)
    dW2 = plan_uv.adjoint(U, V, idx, g)
    torch.cuda.synchronize()
    idx_np, g_np = to_np(idx), to_np(g).astype(np.float64)
    for li, l in enumerate(layers):
        W64 = Ws[li].astype(np.float64)
        ref = oracle.sigma_grad(W64, l.n, l.m, idx_np[li], g_np[li])
        for tag, d in (("plain", dW), ("adjoint", dW2), ("persistent", dWp)):
            _grad_check(W64, l, idx_np[li], g_np[li], d[li], f"layer {li} {tag}", ref)


def test_sigma_topk_autograd_finite_differences():
    """d(sum of top-8 sigma per layer)/dW through the autograd Function,
    against central finite differences of the FP64 oracle's loss."""
    banner("autograd FD")
    layers, Ws = _small_stack(seed=13)
    layers, Ws = layers[:4], Ws[:4]
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs)
    Wt = [_w(W).requires_grad_(True) for W in Ws]
    vals, idx = lfa().sigma_topk(plan, Wt, 8)
    vals.sum().backward()
    rng = np.random.default_rng(1)
    for li, l in enumerate(layers):
        W64 = Ws[li].astype(np.float64)

        def loss(Wx):
            s = oracle.lfa_svd(Wx, l.n, l.m)
            return np.sum(np.sort(s.ravel())[::-1][:8])

        D = rng.standard_normal(W64.shape)
        h = 1e-4 * np.linalg.norm(W64) / np.linalg.norm(D)
        fd = (loss(W64 + h * D) - loss(W64 - h * D)) / (2 * h)
        an = float(np.sum(to_np(Wt[li].grad).astype(np.float64) * D))
        assert abs(fd - an) <= 1e-3 * max(abs(fd), 1e-12), (li, fd, an)


def test_graph_replay_matches_eager():
    banner("graph replay")
    layers, Ws = _small_stack(seed=21)
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs)
    Wt = [_w(W) for W in Ws]
    step = lfa().GraphStep(plan, Wt, 8)
    rng = np.random.default_rng(5)
    for rep in range(3):
        for W in Wt:
            W.copy_(torch.from_numpy(rng.standard_normal(tuple(W.shape)).astype(np.float32) * 0.1))
        st = step.replay()
        st.synchronize()
        S, _, _, _ = plan.svd(Wt, persistent=False)
        vals, idx = plan.topk(S, 8)
        dW = plan.sigma_grad(Wt, idx, torch.ones(len(specs), 8, device=DEV))
        torch.cuda.synchronize()
        np.testing.assert_allclose(to_np(step.vals), to_np(vals), rtol=1e-5)
        idx_g = to_np(step.idx)
        for li, l in enumerate(layers):
            W64 = to_np(Wt[li]).astype(np.float64)
            _grad_check(W64, l, idx_g[li], np.ones(8), step.dW[li], f"replay {rep} layer {li} graph")
            _grad_check(W64, l, to_np(idx)[li], np.ones(8), dW[li], f"replay {rep} layer {li} eager")


def test_graph_with_vectors_replay_matches_eager():
    """The graph that keeps every symbol's U and V (lfa_graph_create_uv):
    three replays with new weights in between, each against the eager
    sigma-only path (sigma, top-8 values, and dW from the recomputed
    vectors of the picks)."""
    banner("graph replay with vectors")
    layers, Ws = _small_stack(seed=23)
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs)
    plan_uv = lfa().Plan(specs, want_u=True, want_v=True)
    Wt = [_w(W) for W in Ws]
    step = lfa().GraphStep(plan_uv, Wt, 8)
    rng = np.random.default_rng(6)
    for rep in range(3):
        for W in Wt:
            W.copy_(torch.from_numpy(rng.standard_normal(tuple(W.shape)).astype(np.float32) * 0.1))
        st = step.replay()
        st.synchronize()
        S, _, _, _ = plan.svd(Wt, persistent=False)
        vals, idx = plan.topk(S, 8)
        dW = plan.sigma_grad(Wt, idx, torch.ones(len(specs), 8, device=DEV))
        torch.cuda.synchronize()
        for a, b in zip(step.S, S):
            np.testing.assert_allclose(to_np(a), to_np(b), rtol=1e-5, atol=1e-6 * float(b.max()))
        np.testing.assert_allclose(to_np(step.vals), to_np(vals), rtol=1e-5)
        idx_g = to_np(step.idx)
        for li, l in enumerate(layers):
            W64 = to_np(Wt[li]).astype(np.float64)
            _grad_check(W64, l, idx_g[li], np.ones(8), step.dW[li], f"uv replay {rep} layer {li} graph")
            _grad_check(W64, l, to_np(idx)[li], np.ones(8), dW[li], f"uv replay {rep} layer {li} eager")


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("persistent", [False, True])
def test_onesided_adjoint_matches_oracle(wide, persistent):
    """Forward pass keeping only the accumulator-free side (U of tall layers,
    V of wide ones), top-8, and lfa_adjoint_onesided (the other side of
    each pick recomputed from W): dW against the oracle's gradient for the
    same picks (elementwise for separated picks) and against the full
    adjoint of a plan keeping both sides."""
    banner(f"one-sided adjoint wide={wide} persistent={persistent}")
    shapes = ((3, 16, 8), (16, 64, 6), (64, 96, 4), (96, 160, 3))
    if wide:
        shapes = tuple((co, ci, n) for ci, co, n in shapes)
    layers, Ws = workloads.resnet18_stack(seed=27, shapes=shapes)
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs, want_u=not wide, want_v=wide)
    Wt = [_w(W) for W in Ws]
    S, U, V, info = plan.svd(Wt, persistent=persistent)
    X = V if wide else U
    vals, idx = plan.topk(S, 8)
    g = torch.linspace(0.5, 1.5, 8, device=DEV).repeat(len(layers), 1)
    dW = plan.adjoint_onesided(Wt, S, X, idx, g)
    plan_uv = lfa().Plan(specs, want_u=True, want_v=True)
    _, U2, V2, _ = plan_uv.svd(Wt)
    dW2 = plan_uv.adjoint(U2, V2, idx, g)
    torch.cuda.synchronize()
    assert plan.info_status(info) == 0
    idx_np, g_np = to_np(idx), to_np(g).astype(np.float64)
    for li, l in enumerate(layers):
        W64 = Ws[li].astype(np.float64)
        ref = oracle.sigma_grad(W64, l.n, l.m, idx_np[li], g_np[li])
        _grad_check(W64, l, idx_np[li], g_np[li], dW[li], f"one-sided layer {li}", ref)
        _grad_check(W64, l, idx_np[li], g_np[li], dW2[li], f"two-sided layer {li}", ref)


def test_onesided_graph_replay_matches_oracle():
    """lfa_graph_create_onesided: three replays with new weights and eager
    work in between; each replay's top-8 values against the oracle's
    spectrum and its dW against the oracle's gradient for its picks."""
    banner("one-sided graph replay")
    layers, Ws = _small_stack(seed=29)
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs, want_u=True)
    Wt = [_w(W) for W in Ws]
    step = lfa().GraphStep(plan, Wt, 8)
    rng = np.random.default_rng(30)
    for rep in range(3):
        news = [(rng.standard_normal(W.shape) * 0.1).astype(np.float32) for W in Ws]
        for W, x in zip(Wt, news):
            W.copy_(torch.from_numpy(x))
        step.replay().synchronize()
        assert plan.info_status(step.info) == 0
        v, ix = to_np(step.vals), to_np(step.idx)
        for li, l in enumerate(layers):
            W64 = news[li].astype(np.float64)
            s_ref = oracle.lfa_svd(W64, l.n, l.m)
            ov, _ = oracle.topk(s_ref, 8)
            np.testing.assert_allclose(v[li], ov, rtol=0, atol=1e-5 * ov[0])
            _grad_check(W64, l, ix[li], np.ones(8), step.dW[li], f"one-sided replay {rep} layer {li}")
        plan.topk(step.S, 8)
        torch.cuda.synchronize()


# ------------------------------------------------- spectral functions --

APPLY_GPU_CASES = [
    # c_out, c_in, n, m, batch, dtype
    (16, 16, 8, 8, 3, np.float32),
    (24, 40, 6, 10, 2, np.float32),     # c_out < c_in
    (40, 24, 7, 5, 2, np.float32),      # odd grid
    (64, 64, 8, 8, 2, np.float32),
    (12, 8, 6, 4, 2, np.float64),
    (12, 8, 8, 8, 2, np.float64),       # in-LDS FFT on both axes, FP64
]

# Larger power-of-two axes (the in-LDS FFT with several lines, or one
# 512- or 1024-point line, per work-group); their spectra have no gap for a
# cut-off level, so only the operator itself is applied.
APPLY_FFT_CASES = [
    (8, 8, 64, 32, 2, np.float32),
    (4, 4, 512, 4, 1, np.float32),
    (6, 4, 1024, 4, 1, np.float64),
    (4, 4, 1024, 8, 1, np.float32),
]


def _gap_level(S, frac):
    """A level near frac * sigma_max in a gap of the spectrum, at least
    1e-3 sigma_max from every singular value (a cut-off on a singular value
    would decide by rounding)."""
    s = np.sort(S.ravel())
    tgt = frac * s[-1]
    gaps = np.where(np.diff(s) > 2e-3 * s[-1])[0]
    i = gaps[np.argmin(np.abs(s[gaps] - tgt))]
    return 0.5 * (s[i] + s[i + 1])


@pytest.mark.parametrize("case,kind", [(c, k) for c in APPLY_GPU_CASES
                                        for k in ("identity", "clip", "truncate", "pinv")]
                         + [(c, "identity") for c in APPLY_FFT_CASES])
def test_apply_matches_oracle(case, kind):
    """lfa_apply (transforms, per-frequency spectral map, inverse transforms)
    on the GPU's own SVD, against the oracle's spectral function of the same
    weights.  Gates: FP32 5e-5 of max|y| (1e-3 for the pseudo-inverse, whose
    cut-off at ~0.1 sigma_max amplifies the SVD's errors up to 10x); FP64
    1e-10."""
    c_out, c_in, n, m, B, dt = case
    banner(f"apply {kind} {case}")
    _, W = workloads.random_layer(c_out, c_in, 3, 3, n, m, seed=41, dtype=dt)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    plan = lfa().Plan([lfa().LayerSpec(c_out, c_in, 3, 3, n, m)], tdt, True, True)
    S, U, V, info = plan.svd([_w(W)])
    S_ref = oracle.lfa_svd(W.astype(np.float64), n, m)
    param = 0.0
    if kind in ("clip", "truncate"):
        param = _gap_level(S_ref, 0.5)
    if kind == "pinv":
        param = _gap_level(S_ref, 0.1)
    cx = c_out if kind == "pinv" else c_in
    rng = np.random.default_rng(42)
    x = rng.standard_normal((B, cx, n, m)).astype(dt)
    y = plan.apply(0, S[0], U[0], V[0], _w(x), kind, param)
    torch.cuda.synchronize()
    ref = oracle.apply_spectral(W.astype(np.float64), x.astype(np.float64), n, m, kind, param)
    err = np.max(np.abs(to_np(y) - ref)) / np.max(np.abs(ref))
    gate = (1e-3 if kind == "pinv" else 5e-5) if dt == np.float32 else 1e-10
    assert err <= gate, f"{kind} {case}: {err:.3e}"


def test_apply_pinv_round_trip_and_batch_independence():
    """Pseudo-inverse after the operator returns the input (square, full
    rank, no cut-off), and every image of a batch comes out as it would
    alone."""
    banner("apply round trip")
    n = m = 8
    _, W = workloads.random_layer(16, 16, 3, 3, n, m, seed=43, dtype=np.float64)
    plan = lfa().Plan([lfa().LayerSpec(16, 16, 3, 3, n, m)], torch.float64, True, True)
    S, U, V, info = plan.svd([_w(W)])
    smin, smax = float(S[0].min()), float(S[0].max())
    assert smin > 1e-3 * smax
    rng = np.random.default_rng(44)
    x = _w(rng.standard_normal((3, 16, n, m)))
    Ax = plan.apply(0, S[0], U[0], V[0], x, "identity")
    back = plan.apply(0, S[0], U[0], V[0], Ax, "pinv", 0.0)
    torch.cuda.synchronize()
    assert float((back - x).abs().max()) <= 1e-12 * float(x.abs().max()) * smax / smin
    one = plan.apply(0, S[0], U[0], V[0], x[1:2].contiguous(), "identity")
    assert torch.equal(one[0], Ax[1])


# ---------------------------------------------------------------- lift --

LIFT_CASES = [
    # c_out, c_in, n, m, dtype
    (16, 16, 8, 8, np.float32),
    (24, 40, 6, 10, np.float32),
    (12, 8, 7, 5, np.float64),
]


@pytest.mark.parametrize("case", LIFT_CASES)
def test_lift_matches_oracle_and_maps_v_to_sigma_u(case):
    """lfa_lift against the oracle's lift (Fourier basis times the symbol's
    singular vectors) of the same U, V columns, for the layer's top-k picks
    plus a conjugate-side pick and an out-of-range one; the lifted vectors
    have unit norm and the operator (lfa_apply, identity, on the real and
    imaginary parts) maps v_hat to sigma u_hat."""
    c_out, c_in, n, m, dt = case
    banner(f"lift {case}")
    _, W = workloads.random_layer(c_out, c_in, 3, 3, n, m, seed=45, dtype=dt)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    plan = lfa().Plan([lfa().LayerSpec(c_out, c_in, 3, 3, n, m)], tdt, True, True)
    S, U, V, info = plan.svd([_w(W)])
    vals, idx = plan.topk(S, 4)
    picks = torch.cat([idx[0], torch.tensor([[n - 1, m - 1, 1], [n, 0, 0]], dtype=torch.int32, device=DEV)])
    uh, vh = plan.lift(0, U[0], V[0], picks.contiguous())
    torch.cuda.synchronize()
    Un, Vn, Sn = to_np(U[0]).astype(np.complex128), to_np(V[0]).astype(np.complex128), to_np(S[0])
    pk = picks.cpu().numpy()
    tol = 2e-6 if dt == np.float32 else 1e-13
    for t in range(len(pk) - 1):
        p, q, j = (int(v) for v in pk[t])
        Uo, Vo = oracle.lift(Un[p, q], Vn[p, q], n, m, p, q)      # [(x1 m + x2) c + ch, r]
        uo = Uo[:, j].reshape(n, m, c_out).transpose(2, 0, 1)
        vo = Vo[:, j].reshape(n, m, c_in).transpose(2, 0, 1)
        ug, vg = to_np(uh[t]), to_np(vh[t])
        assert np.max(np.abs(ug - uo)) <= tol * np.max(np.abs(uo)), (t, p, q, j)
        assert np.max(np.abs(vg - vo)) <= tol * np.max(np.abs(vo)), (t, p, q, j)
        assert abs(np.linalg.norm(ug) - 1.0) <= 1e-5 and abs(np.linalg.norm(vg) - 1.0) <= 1e-5
    assert float(uh[-1].abs().max()) == 0.0 and float(vh[-1].abs().max()) == 0.0
    # the operator maps v_hat to sigma u_hat (apply is real-linear)
    count = len(pk) - 1
    xr = vh[:count].real.contiguous()
    xi = vh[:count].imag.contiguous()
    yr = plan.apply(0, S[0], U[0], V[0], xr, "identity")
    yi = plan.apply(0, S[0], U[0], V[0], xi, "identity")
    torch.cuda.synchronize()
    Av = to_np(yr).astype(np.complex128) + 1j * to_np(yi)
    for t in range(count):
        p, q, j = (int(v) for v in pk[t])
        su = Sn[p, q, j] * to_np(uh[t])
        gate = (5e-5 if dt == np.float32 else 1e-11) * float(Sn.max())
        assert np.max(np.abs(Av[t] - su)) <= gate * np.max(np.abs(to_np(uh[t]))), (t, p, q, j)
    # one output only
    only_u, none_v = plan.lift(0, U[0], None, picks[:2].contiguous())
    torch.cuda.synchronize()
    assert none_v is None and torch.equal(only_u, uh[:2])


# ---------------------------------------------------------------- crystals --

CRYSTAL_CASES = [
    # c_out, c_in, kh, kw, n, m, stride, dtype
    (16, 8, 3, 3, 16, 16, 2, np.float32),       # 3x3 stride 2 (downsampling)
    (32, 3, 7, 7, 32, 32, 2, np.float32),       # 7x7 stride 2 stem
    (24, 16, 1, 1, 12, 8, 2, np.float32),       # 1x1 stride-2 shortcut
    (8, 4, 3, 3, 18, 12, 3, np.float32),
    (12, 6, 4, 4, 16, 16, 2, np.float64),       # even extent
    (64, 16, 3, 3, 16, 16, 2, np.float32),      # 64 x 64 symbols
]


def _crystal(case):
    c_out, c_in, kh, kw, n, m, s, dt = case
    spec = lfa().LayerSpec(c_out, c_in, kh, kw, n, m)
    rng = np.random.default_rng(61)
    W = (rng.standard_normal((c_out, c_in, kh, kw)) / np.sqrt(c_in * kh * kw)).astype(dt)
    return spec, s, W, lfa().crystal_layer(spec, s)


@pytest.mark.parametrize("case", CRYSTAL_CASES)
def test_crystal_symbols_and_sigma_match_oracle(case):
    """A strided layer through its crystal form: lfa_crystal_weights, then
    the stride-1 symbols and SVD of the coarse layer, against the oracle's
    crystal symbols (defined from the strided operator, not from a repack)
    and their LAPACK SVD.  Symbols within 1e-6 (FP32) / 1e-13 (FP64) of their
    largest entry; sigma within the usual gates; the adjoint repack returns W."""
    spec, s, W, c = _crystal(case)
    banner(f"crystal {case}")
    tdt = torch.float32 if W.dtype == np.float32 else torch.float64
    Wc = lfa().crystal_weights(_w(W), spec, s)
    A = lfa().symbols(Wc, c.n, c.m)
    back = lfa().crystal_weights(Wc, spec, s, adjoint=True)
    torch.cuda.synchronize()
    assert torch.equal(back, _w(W))
    A_ref = oracle.crystal_symbols(W.astype(np.float64), spec.n, spec.m, s)
    tol = 1e-6 if tdt == torch.float32 else 1e-13
    assert np.max(np.abs(to_np(A) - A_ref)) <= tol * np.max(np.abs(A_ref))
    S = lfa().svd(Wc, c.n, c.m)
    torch.cuda.synchronize()
    S_ref = np.linalg.svd(A_ref, compute_uv=False)
    e = oracle.sigma_error(to_np(S), S_ref)
    assert e <= sigma_gate(tdt), f"{case}: sigma error {e:.3e}"


def test_crystal_sigma_grad_matches_finite_differences():
    """Gradient of the sum of a strided layer's top-4 singular values: the
    coarse layer's adjoint kernel (lfa_sigma_grad on the crystal weights),
    pulled back to W by the adjoint repack, against central differences of
    the oracle's crystal-symbol singular values at the same picks (FP64)."""
    case = (8, 4, 3, 3, 12, 12, 2, np.float64)
    spec, s, W, c = _crystal(case)
    banner(f"crystal grad {case}")
    plan = lfa().Plan([c], torch.float64, True, True)
    Wc = lfa().crystal_weights(_w(W), spec, s)
    S, _, _, _ = plan.svd([Wc])
    vals, idx = plan.topk(S, 4)
    grad = torch.ones(1, 4, dtype=torch.float64, device=DEV)
    dWc = plan.sigma_grad([Wc], idx, grad)[0]
    dW = to_np(lfa().crystal_weights(dWc.contiguous(), spec, s, adjoint=True))
    torch.cuda.synchronize()
    picks = idx[0].cpu().numpy()

    def loss(Wx):
        A = oracle.crystal_symbols(Wx, spec.n, spec.m, s)
        Sx = np.linalg.svd(A, compute_uv=False)
        return sum(Sx[p, q, j] for p, q, j in picks)

    rng = np.random.default_rng(62)
    for _ in range(3):
        D = rng.standard_normal(W.shape)
        h = 1e-6 * np.linalg.norm(W) / np.linalg.norm(D)
        fd = (loss(W + h * D) - loss(W - h * D)) / (2 * h)
        an = float(np.sum(dW * D))
        assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd)), (an, fd)


QR_CASES = [
    # c_out, c_in, kh, n, m: FP32 sigma-only layers the plan runs through QR
    # preconditioning (working matrix M x N with M > 64 and 4 M >= 5 N)
    (160, 96, 3, 4, 5),       # blocked kernel on the 96 x 96 factors
    (96, 160, 3, 5, 4),       # wide: G = A^H, factors of A A^H
    (128, 64, 3, 6, 6),       # 64 x 64 factors: the register kernel
    (512, 256, 3, 4, 4),      # the rectangular layer's shape on a small grid
    (200, 24, 1, 3, 7),       # 1x1 kernel, odd grid
    (100, 72, 4, 5, 6),       # 16 taps: rows of W not staged in LDS
    (144, 80, 5, 6, 5),       # 25 taps
]


@pytest.mark.parametrize("case", QR_CASES)
def test_qr_preconditioned_vectors_match_oracle(case, monkeypatch):
    """Sigma, U and V of tall FP32 layers through QR preconditioning (the
    SVD of the factors keeps V, the left vectors come from G V): sigma over
    the whole grid, residual and orthonormality on sampled symbols, and the
    gauge-free projectors u_j v_j^H of separated singular values against the
    oracle's."""
    c_out, c_in, kh, n, m = case
    banner(f"qr vectors {case}")
    L, W = workloads.random_layer(c_out, c_in, kh, kh, n, m, seed=52)
    spec = lfa().LayerSpec(c_out, c_in, kh, kh, n, m)
    monkeypatch.setenv("LFA_QR", "1")
    plan = lfa().Plan([spec], want_u=True, want_v=True)
    assert plan.preconditioned(0)
    S, U, V, info = plan.svd([_w(W)])
    torch.cuda.synchronize()
    assert plan.info_status(info) == 0
    S_ref = oracle.lfa_svd(W.astype(np.float64), n, m)
    assert oracle.sigma_error(to_np(S[0]), S_ref) <= 1e-5
    fr = _sample(n, m, 6, 53)
    A = oracle.symbols(W.astype(np.float64), n, m, fr)
    Sg, Ug, Vg = (to_np(x)[fr[:, 0], fr[:, 1]] for x in (S[0], U[0], V[0]))
    check_vectors(A, Sg, Ug, Vg, torch.float32, f"qr {case}")
    s_r, u_r, v_r = oracle.svd_symbols(A)
    check_projectors(s_r, u_r, v_r, Ug, Vg, torch.float32, f"qr {case}")


@pytest.mark.parametrize("case", QR_CASES)
def test_qr_preconditioned_sigma_matches_oracle(case, monkeypatch):
    """Sigma of tall FP32 layers through the Gram-taps Cholesky factors
    (QR preconditioning) against the oracle over the whole grid, and against
    the same plan without preconditioning (LFA_QR=0, read at plan
    creation); Parseval over the whole grid."""
    c_out, c_in, kh, n, m = case
    banner(f"qr {case}")
    L, W = workloads.random_layer(c_out, c_in, kh, kh, n, m, seed=51)
    spec = lfa().LayerSpec(c_out, c_in, kh, kh, n, m)
    monkeypatch.setenv("LFA_QR", "1")
    plan = lfa().Plan([spec])
    assert plan.preconditioned(0)
    S, info = (lambda r: (r[0][0], r[3]))(plan.svd([_w(W)]))
    monkeypatch.setenv("LFA_QR", "0")
    plan2 = lfa().Plan([spec])
    assert not plan2.preconditioned(0)
    S2 = plan2.svd([_w(W)])[0][0]
    torch.cuda.synchronize()
    assert lfa().Plan([spec]).info_status(info) == 0
    S_ref = oracle.lfa_svd(W.astype(np.float64), n, m)
    e1 = oracle.sigma_error(to_np(S), S_ref)
    e2 = oracle.sigma_error(to_np(S2), S_ref)
    print(f"[qr] {case}: error with QR {e1:.2e}, without {e2:.2e}", flush=True)
    assert e1 <= 1e-5 and e2 <= 1e-5
    ss = torch.sum(S.double() ** 2).item()
    assert abs(ss / (n * m * np.sum(W.astype(np.float64) ** 2)) - 1) <= 1e-5


def test_qr_preconditioned_rank_deficient_zeros(monkeypatch):
    """Rank-one taps (rank <= 9 per symbol) through QR preconditioning: the
    numerically singular pivots give zero rows of R, and the singular values
    beyond the rank come out exactly 0; the others match the oracle."""
    banner("qr rank-one")
    L, W = workloads.rank_one_taps(c_out=192, c_in=96, n=4)
    spec = lfa().LayerSpec(L.c_out, L.c_in, L.kh, L.kw, L.n, L.m)
    monkeypatch.setenv("LFA_QR", "1")
    plan = lfa().Plan([spec])
    assert plan.preconditioned(0)
    S = plan.svd([_w(W)])[0][0]
    torch.cuda.synchronize()
    S_ref = oracle.lfa_svd(W.astype(np.float64), L.n, L.m)
    assert oracle.sigma_error(to_np(S), S_ref) <= 1e-5
    assert np.all(to_np(S)[..., 9:] == 0)


GRADED_CASES = [
    # c_out, c_in, kh, n, m, LFA_QR: tall FP32 layers, input channels scaled
    # by 1, 10^2.5, 10^5 in turn
    (64, 48, 3, 4, 4, "0"),       # register kernel
    (160, 96, 3, 3, 3, "0"),      # blocked kernel
    (160, 96, 3, 3, 3, "1"),      # QR preconditioning, left vectors from G V
]


@pytest.mark.parametrize("case", GRADED_CASES)
def test_graded_columns_relative_accuracy(case, monkeypatch):
    """Symbols with columns graded over five decades.  One-sided Jacobi with
    a threshold relative to the two columns' norms finds even the smallest
    singular values to a relative accuracy set by the condition of the
    column-normalised matrix (here about 1e-5 in FP32), where an algorithm
    accurate only normwise would err by u sigma_max / sigma, up to 1e-1.
    Every singular value of the grid against the oracle's, relative to
    itself (gate 1e-4); orthonormality of U and V and the residual on
    sampled symbols; projectors of separated values."""
    c_out, c_in, kh, n, m, qr = case
    banner(f"graded {case}")
    L, W = workloads.graded_channels(c_out, c_in, kh, kh, n, m, seed=57)
    spec = lfa().LayerSpec(c_out, c_in, kh, kh, n, m)
    monkeypatch.setenv("LFA_QR", qr)
    plan = lfa().Plan([spec], want_u=True, want_v=True)
    assert plan.preconditioned(0) == (qr == "1")
    S, U, V, info = plan.svd([_w(W)])
    torch.cuda.synchronize()
    assert plan.info_status(info) == 0
    W64 = W.astype(np.float64)
    S_ref = oracle.lfa_svd(W64, n, m)
    Sg = to_np(S[0]).astype(np.float64)
    assert S_ref.min() > 0 and S_ref.max() / S_ref.min() > 1e4
    rel = float(np.max(np.abs(Sg - S_ref) / S_ref))
    print(f"[graded] {case}: max relative sigma error {rel:.2e}, "
          f"range {S_ref.max() / S_ref.min():.1e}", flush=True)
    assert rel <= 1e-4, f"{case}: relative sigma error {rel:.3e}"
    fr = _sample(n, m, 4, 58)
    A = oracle.symbols(W64, n, m, fr)
    Sg, Ug, Vg = (to_np(x)[fr[:, 0], fr[:, 1]] for x in (S[0], U[0], V[0]))
    check_vectors(A, Sg, Ug, Vg, torch.float32, f"graded {case}")
    s_r, u_r, v_r = oracle.svd_symbols(A)
    check_projectors(s_r, u_r, v_r, Ug, Vg, torch.float32, f"graded {case}")


DUAL_CASES = [
    # c_out, c_in, kh, n, m, vectors: more than 256 canonical symbols of more
    # than 64 rows, so the blocked kernel runs without teams and takes two
    # block pairs per cross step (LFA_QR=0)
    (160, 96, 1, 24, 24, False),    # 6 column blocks: 3 pairs per outer step, one step with one pair
    (224, 200, 1, 24, 24, False),   # 13 blocks, the last one partial (8 columns), a padded block
    (160, 96, 1, 24, 24, True),     # U only: the accumulator-free side, still dual
]


@pytest.mark.parametrize("case", DUAL_CASES)
def test_blocked_dual_cross_steps(case, monkeypatch):
    """The blocked kernel's dual cross steps (two block pairs per step) with
    an odd number of block pairs per outer step and a partial last block:
    sigma over the whole grid against the oracle; with U, orthonormality of
    U and, gauge-free, (A^H U)^H (A^H U) = S^2 on sampled symbols."""
    c_out, c_in, kh, n, m, vectors = case
    banner(f"dual {case}")
    L, W = workloads.random_layer(c_out, c_in, kh, kh, n, m, seed=59)
    spec = lfa().LayerSpec(c_out, c_in, kh, kh, n, m)
    monkeypatch.setenv("LFA_QR", "0")
    plan = lfa().Plan([spec], want_u=vectors)
    assert not plan.preconditioned(0)
    S, U, V, info = plan.svd([_w(W)])
    torch.cuda.synchronize()
    assert plan.info_status(info) == 0
    W64 = W.astype(np.float64)
    S_ref = oracle.lfa_svd(W64, n, m)
    e = oracle.sigma_error(to_np(S[0]), S_ref)
    print(f"[dual] {case}: sigma error {e:.2e}", flush=True)
    assert e <= 1e-5
    if vectors:
        fr = _sample(n, m, 6, 60)
        A = oracle.symbols(W64, n, m, fr)
        Sg = to_np(S[0])[fr[:, 0], fr[:, 1]].astype(np.float64)
        Ug = to_np(U[0])[fr[:, 0], fr[:, 1]].astype(np.complex128)
        r = Sg.shape[-1]
        ou = np.max(np.abs(np.conj(np.swapaxes(Ug, -1, -2)) @ Ug - np.eye(r)))
        assert ou <= 1e-5, f"U orthonormality {ou:.3e}"
        X = np.conj(np.swapaxes(A, -1, -2)) @ Ug                       # A^H U = V S
        Gm = np.conj(np.swapaxes(X, -1, -2)) @ X
        D = np.zeros_like(Gm)
        idx = np.arange(r)
        D[..., idx, idx] = Sg ** 2
        err = np.max(np.abs(Gm - D)) / np.max(Sg[..., 0]) ** 2
        assert err <= 1e-5, f"(A^H U)^H (A^H U) - S^2: {err:.3e}"


# ------------------------------------------------- rank-deficient symbols --

RANK_DEFICIENT_CASES = [
    # c_out, c_in, kh, n, m, z (channels of the long side kept), dtype, vectors
    (64, 24, 1, 6, 4, 16, np.float32, False),     # register kernel, NC 32 > N 24
    (64, 24, 1, 6, 4, 16, np.float32, True),
    (24, 64, 3, 6, 4, 16, np.float32, False),     # wide (G = A^H)
    (64, 24, 1, 6, 4, 16, np.float64, True),
    (160, 96, 1, 4, 4, 40, np.float32, True),     # blocked kernel, rank 40 of 96
    (160, 96, 1, 4, 4, 40, np.float64, False),
]


@pytest.mark.parametrize("case", RANK_DEFICIENT_CASES)
def test_rank_deficient_symbols_converge(case):
    """Symbols of rank z below their column count (the channels past z on the
    long side of the symbol are zero: zero rows of the working matrix, whose
    columns then span z dimensions only): every symbol converges in a normal
    number of sweeps, sigma is finite and within the gate, the missing
    singular values are exactly 0, and with vectors U and V are orthonormal
    (zero columns completed).  Regression: the noise left in the vanishing
    columns used to be rotated until it underflowed (FP32 turned it into
    NaN; FP64 ran to the sweep limit)."""
    c_out, c_in, kh, n, m, z, dt, vec = case
    banner(f"rank-deficient {case}")
    rng = np.random.default_rng(71)
    W = (rng.standard_normal((c_out, c_in, kh, kh)) / np.sqrt(c_in * kh * kh)).astype(dt)
    if c_out >= c_in:
        W[z:, :] = 0
    else:
        W[:, z:] = 0
    tdt = torch.float32 if dt == np.float32 else torch.float64
    plan = lfa().Plan([lfa().LayerSpec(c_out, c_in, kh, kh, n, m)], tdt, vec, vec)
    S, U, V, info = plan.svd([_w(W)])
    torch.cuda.synchronize()
    info = to_np(info[0])
    S = to_np(S[0])
    assert np.all(np.isfinite(S)) and info[lfa()._lib.LFA_INFO_NONFINITE] == 0
    # the vanishing columns shrink geometrically (by about 5x per sweep in the
    # blocked kernel's block order: about 12 sweeps in FP32 and 24 in FP64
    # for these shapes, matching a CPU emulation of that order; 8 to 11 in
    # the register kernel); the limit is 40
    limit = 16 if dt == np.float32 else 30
    assert info[lfa()._lib.LFA_INFO_NONCONVERGED] == 0 and info[lfa()._lib.LFA_INFO_MAX_SWEEPS] <= limit, info
    A = oracle.symbols(W.astype(np.float64), n, m)
    S_ref = oracle.svd_symbols(A, compute_uv=False)
    assert oracle.sigma_error(S, S_ref) <= sigma_gate(tdt)
    assert np.all(S[..., z:] == 0)
    if vec:
        check_vectors(A, S, to_np(U[0]), to_np(V[0]), tdt, "rank-deficient")


def test_crystal_apply_is_the_strided_convolution():
    """The spectral apply (identity) of a stride-2 layer's crystal form, on
    the input rearranged into the crystal's channels (torch's
    pixel_unshuffle: point d of a cell is channel i*4 + d1*2 + d2), is the
    strided convolution itself: the oracle's dense strided operator applied
    to the same images."""
    c_out, c_in, k, n, s, B = 16, 6, 3, 16, 2, 2
    banner("crystal apply = strided conv")
    rng = np.random.default_rng(63)
    W = (rng.standard_normal((c_out, c_in, k, k)) / np.sqrt(c_in * k * k)).astype(np.float32)
    spec = lfa().LayerSpec(c_out, c_in, k, k, n, n)
    c = lfa().crystal_layer(spec, s)
    plan = lfa().Plan([c], torch.float32, True, True)
    Wc = lfa().crystal_weights(_w(W), spec, s)
    S, U, V, _ = plan.svd([Wc])
    x = rng.standard_normal((B, c_in, n, n)).astype(np.float32)
    xc = torch.nn.functional.pixel_unshuffle(_w(x), s).contiguous()
    y = plan.apply(0, S[0], U[0], V[0], xc, "identity")
    torch.cuda.synchronize()
    D = oracle.strided_operator(W.astype(np.float64), n, n, s)
    xv = np.transpose(x.astype(np.float64), (0, 2, 3, 1)).reshape(B, -1)       # (z1 n + z2) c_in + i
    ref = np.transpose((xv @ D.T).reshape(B, n // s, n // s, c_out), (0, 3, 1, 2))
    err = np.max(np.abs(to_np(y) - ref)) / np.max(np.abs(ref))
    assert err <= 5e-5, err


# -------------------------------------------- the other workloads, full size --

def _sample(n, m, count, seed):
    rng = np.random.default_rng(seed)
    fr = np.stack([rng.integers(0, n, count), rng.integers(0, m, count)], axis=1)
    fr[0] = (0, 0)
    fr[1] = (n - 1, m - 1)
    return fr


@pytest.mark.parametrize("vectors", [False, True])
def test_rectangular_512x256_full_size_sampled(vectors):
    """256 -> 512 channels, 3x3, 32x32 grid (1024 symbols of 512 x 256), in
    the benchmark's launch configuration: 12 sampled symbols and the last
    canonical ones against the oracle (sigma; with vectors also residual,
    orthonormality and projectors), Parseval over the whole grid."""
    banner(f"512x256 full size, vectors={vectors}")
    L, W = workloads.rectangular_256_512()
    out, info = lfa().svd(_w(W), L.n, L.m, compute_uv=vectors, return_info=True)
    torch.cuda.synchronize()
    S = out[0] if vectors else out
    assert info[0] == 0 and info[3] == 0, info
    # plus the last canonical frequencies (row n/2 of the grid, up to m/2),
    # which the teams of the short last round decompose, and a mirror
    fr = np.concatenate([_sample(L.n, L.m, 12, 5),
                         [[L.n // 2, L.m // 2 - 1], [L.n // 2, L.m // 2], [L.n // 2, L.m // 2 + 1]]])
    A = oracle.symbols(W.astype(np.float64), L.n, L.m, fr)
    S_ref, U_ref, V_ref = oracle.svd_symbols(A, compute_uv=True)
    Sg = to_np(S)[fr[:, 0], fr[:, 1]]
    assert oracle.sigma_error(Sg, S_ref) <= 1e-5
    if vectors:
        Ug, Vg = to_np(out[1])[fr[:, 0], fr[:, 1]], to_np(out[2])[fr[:, 0], fr[:, 1]]
        check_vectors(A, Sg, Ug, Vg, torch.float32, "512x256")
        check_projectors(S_ref, U_ref, V_ref, Ug, Vg, torch.float32, "512x256")
    ss = torch.sum(S.double() ** 2).item()
    assert abs(ss / (L.n * L.m * np.sum(W.astype(np.float64) ** 2)) - 1) <= 1e-5


def test_blocked_last_round_teams_with_vectors(monkeypatch):
    """The short last round of the blocked kernel with the rotation
    accumulator (vectors, QR preconditioning off): 514 canonical symbols of
    256 x 192, two more than a round of resident work-groups (one or two per
    CU), so the last two run in teams at the end of the same grid.  Sampled
    symbols, the last canonical ones among them, against the oracle (sigma,
    residual, orthonormality); Parseval over the whole grid."""
    monkeypatch.setenv("LFA_QR", "0")
    banner("blocked last-round teams with vectors, 256x192 on 32x32")
    n = m = 32
    _, W = workloads.random_layer(256, 192, 3, 3, n, m, seed=21, dtype=np.float32)
    plan = lfa().Plan([lfa().LayerSpec(256, 192, 3, 3, n, m)], torch.float32, True, True)
    assert not plan.preconditioned(0)
    S, U, V, info = plan.svd([_w(W)])
    torch.cuda.synchronize()
    info = to_np(info)[0]
    assert info[0] == 0 and info[3] == 0, info
    fr = np.concatenate([_sample(n, m, 6, 8), [[n // 2, m // 2 - 1], [n // 2, m // 2], [n // 2, m // 2 + 1]]])
    A = oracle.symbols(W.astype(np.float64), n, m, fr)
    S_ref = oracle.svd_symbols(A, compute_uv=False)
    Sg = to_np(S[0])[fr[:, 0], fr[:, 1]]
    assert oracle.sigma_error(Sg, S_ref) <= 1e-5
    check_vectors(A, Sg, to_np(U[0])[fr[:, 0], fr[:, 1]], to_np(V[0])[fr[:, 0], fr[:, 1]], torch.float32,
                  "last-round teams")
    ss = torch.sum(S[0].double() ** 2).item()
    assert abs(ss / (n * m * np.sum(W.astype(np.float64) ** 2)) - 1) <= 1e-5


def test_rank_one_512x256_full_size_sampled():
    """The rank-deficient instance at full size (rank-one taps: rank 9 per
    symbol), with vectors: sampled sigma against the oracle, the 247
    vanishing values exactly 0, U and V orthonormal (completed columns
    included), Parseval over the whole grid."""
    banner("rank-one 512x256 full size")
    L, W = workloads.rank_one_taps()
    (S, U, V), info = lfa().svd(_w(W), L.n, L.m, compute_uv=True, return_info=True)
    torch.cuda.synchronize()
    assert info[0] == 0 and info[3] == 0, info
    fr = _sample(L.n, L.m, 8, 6)
    A = oracle.symbols(W.astype(np.float64), L.n, L.m, fr)
    S_ref = oracle.svd_symbols(A, compute_uv=False)
    Sg = to_np(S)[fr[:, 0], fr[:, 1]]
    assert oracle.sigma_error(Sg, S_ref) <= 1e-5
    assert np.all(to_np(S)[..., 9:] == 0)
    check_vectors(A, Sg, to_np(U)[fr[:, 0], fr[:, 1]], to_np(V)[fr[:, 0], fr[:, 1]], torch.float32, "rank-one")
    ss = torch.sum(S.double() ** 2).item()
    assert abs(ss / (L.n * L.m * np.sum(W.astype(np.float64) ** 2)) - 1) <= 1e-5


def test_resnet18_stack_full_size():
    """The twelve ResNet-18 layers at their real grids, as the benchmark's
    batched step runs them: one persistent sigma-only launch, top-8 per
    layer, gradient of the top-8 sum.  Per layer: sampled sigma against the
    oracle, the top-8 values equal to the oracle's singular values at the
    chosen (p, q, j), and dW against the oracle's gradient for those picks."""
    banner("ResNet-18 stack full size")
    layers, Ws = workloads.resnet18_stack()
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs)
    Wt = [_w(W) for W in Ws]
    S, _, _, info = plan.svd(Wt, persistent=True)
    vals, idx = plan.topk(S, 8)
    g = torch.ones(len(layers), 8, device=DEV)
    dW = plan.sigma_grad(Wt, idx, g, persistent=True)
    torch.cuda.synchronize()
    assert int(to_np(info)[:, 0].sum()) == 0
    vals, idx = to_np(vals), to_np(idx)
    for li, l in enumerate(layers):
        W64 = Ws[li].astype(np.float64)
        fr = _sample(l.n, l.m, 6, 20 + li)
        assert oracle.sigma_error(to_np(S[li])[fr[:, 0], fr[:, 1]], oracle.lfa_svd(W64, l.n, l.m, freqs=fr)) <= 1e-5
        p, q, j = idx[li].T
        s_at = oracle.lfa_svd(W64, l.n, l.m, freqs=np.stack([p, q], axis=1))[np.arange(8), j]
        assert np.max(np.abs(vals[li] - s_at)) <= 1e-5 * s_at.max(), li
        _grad_check(W64, l, idx[li], np.ones(8), dW[li], f"full stack layer {li}")


def _oracle_sigma_threaded(W64, n, m, threads=16):
    """The oracle's singular values of every symbol of a layer, frequency
    chunks spread over host threads (numpy's SVD releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    pp, qq = np.meshgrid(np.arange(n), np.arange(m), indexing="ij")
    fr = np.stack([pp.ravel(), qq.ravel()], axis=1)
    chunks = np.array_split(fr, min(len(fr), threads * 4))
    with ThreadPoolExecutor(max_workers=min(threads, os.cpu_count() or 1)) as ex:
        parts = list(ex.map(lambda c: oracle.lfa_svd(W64, n, m, freqs=c), chunks))
    return np.concatenate(parts).reshape(n, m, -1)


def test_resnet18_stack_full_size_finite_differences():
    """The benchmark's gradient at full size: the twelve ResNet-18 layers,
    persistent sigma-only launch, top-8 per layer and the persistent sigma
    gradient, against central finite differences of the oracle's top-8 sum
    of each layer along a random direction (every symbol of the layer
    recomputed in FP64 at W +- h D), at 1e-3 relative."""
    banner("ResNet-18 stack full size, finite differences")
    layers, Ws = workloads.resnet18_stack()
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs)
    Wt = [_w(W).requires_grad_(True) for W in Ws]
    vals, idx = lfa().sigma_topk(plan, Wt, 8)
    vals.sum().backward()
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    for li, l in enumerate(layers):
        W64 = Ws[li].astype(np.float64)

        def loss(Wx):
            s = _oracle_sigma_threaded(Wx, l.n, l.m)
            return float(np.sum(np.sort(s.ravel())[::-1][:8]))

        D = rng.standard_normal(W64.shape)
        h = 1e-7 * np.linalg.norm(W64) / np.linalg.norm(D)
        fd = (loss(W64 + h * D) - loss(W64 - h * D)) / (2 * h)
        an = float(np.sum(to_np(Wt[li].grad).astype(np.float64) * D))
        print(f"[fd] layer {li} fd {fd:.9e} gpu {an:.9e} rel {abs(fd - an) / abs(fd):.2e}", flush=True)
        assert abs(fd - an) <= 1e-3 * abs(fd), (li, fd, an)


def test_resnet18_stack_full_size_vectors_graph():
    """The benchmark's batched step as it runs: one HIP graph of the
    persistent SVD keeping every symbol's U and V, top-8 per layer and one
    adjoint launch, replayed twice with eager work in between.  Each replay:
    top-8 values equal to the oracle's singular values at the chosen
    (p, q, j), and dW against the oracle's gradient for those picks."""
    banner("ResNet-18 stack full size, graph with vectors")
    layers, Ws = workloads.resnet18_stack()
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs, want_u=True, want_v=True)
    Wt = [_w(W) for W in Ws]
    step = lfa().GraphStep(plan, Wt, 8)
    refs = {}
    for rep in range(2):
        step.replay().synchronize()
        assert int(to_np(step.info)[:, 0].sum()) == 0
        vals, idx = to_np(step.vals), to_np(step.idx)
        for li, l in enumerate(layers):
            W64 = Ws[li].astype(np.float64)
            p, q, j = idx[li].T
            s_at = oracle.lfa_svd(W64, l.n, l.m, freqs=np.stack([p, q], axis=1))[np.arange(8), j]
            assert np.max(np.abs(vals[li] - s_at)) <= 1e-5 * s_at.max(), (rep, li)
            key = (li, idx[li].tobytes())
            if key not in refs:
                refs[key] = oracle.sigma_grad(W64, l.n, l.m, idx[li], np.ones(8))
            _grad_check(W64, l, idx[li], np.ones(8), step.dW[li], f"uv graph replay {rep} layer {li}",
                        refs[key])
        # eager work between the replays
        plan.topk(step.S, 8)
        torch.cuda.synchronize()


def test_resnet18_stack_full_size_onesided_graph():
    """The benchmark's batched step: one HIP graph of the persistent SVD
    keeping U of every symbol (no rotation accumulator), top-8 and the
    one-sided adjoint, replayed twice with eager work in between: top-8
    values against the oracle's singular values at the picks, dW against
    the oracle's gradient elementwise, every symbol's sigma within the gate
    on sampled frequencies of each layer."""
    banner("ResNet-18 stack full size, one-sided graph")
    layers, Ws = workloads.resnet18_stack()
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa().Plan(specs, want_u=True)
    Wt = [_w(W) for W in Ws]
    step = lfa().GraphStep(plan, Wt, 8)
    refs = {}
    for rep in range(2):
        step.replay().synchronize()
        assert plan.info_status(step.info) == 0
        vals, idx = to_np(step.vals), to_np(step.idx)
        for li, l in enumerate(layers):
            W64 = Ws[li].astype(np.float64)
            p, q, j = idx[li].T
            s_at = oracle.lfa_svd(W64, l.n, l.m, freqs=np.stack([p, q], axis=1))[np.arange(8), j]
            assert np.max(np.abs(vals[li] - s_at)) <= 1e-5 * s_at.max(), (rep, li)
            key = (li, idx[li].tobytes())
            if key not in refs:
                refs[key] = oracle.sigma_grad(W64, l.n, l.m, idx[li], np.ones(8))
            _grad_check(W64, l, idx[li], np.ones(8), step.dW[li], f"one-sided graph {rep} layer {li}",
                        refs[key])
            if rep == 0:
                fr = _sample(l.n, l.m, 4, 40 + li)
                S_ref = oracle.lfa_svd(W64, l.n, l.m, freqs=fr)
                assert oracle.sigma_error(to_np(step.S[li])[fr[:, 0], fr[:, 1]], S_ref) <= 1e-5
        plan.topk(step.S, 8)
        torch.cuda.synchronize()


def test_autotuned_resnet18_stack_matches_oracle(tmp_path):
    """lfa_autotune on the full ResNet-18 stack (per-layer choices for the
    per-layer SVD, and the persistent launch's cost model) with a JSON
    cache; the tuned plan's one-sided graph step then matches the oracle
    (top-8 values at the picks, dW elementwise, sampled sigma of every
    layer).  A second plan tuned from the same cache gets the same choices
    without timing; the cache is valid JSON with an entry per layer shape and
    one for the persistent launch."""
    import json

    banner("autotuned ResNet-18 stack")
    layers, Ws = workloads.resnet18_stack()
    specs = [lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    Wt = [_w(W) for W in Ws]
    cache = tmp_path / "tune.json"
    plan = lfa().Plan(specs, want_u=True)
    plan.autotune(Wt, cache)
    doc = json.loads(cache.read_text())
    keys = list(doc["entries"])
    assert sum("/layer/" in k for k in keys) == len(set(specs)), keys
    assert sum("/persistent/" in k for k in keys) == 1, keys
    choices = [plan.tuning(i) for i in range(len(specs))]
    print(f"[tune] {choices} cost model {plan.cost_model()}", flush=True)
    plan2 = lfa().Plan(specs, want_u=True)
    import time
    t0 = time.perf_counter()
    plan2.autotune(Wt, cache)
    assert time.perf_counter() - t0 < 2.0
    assert [plan2.tuning(i) for i in range(len(specs))] == choices
    assert plan2.cost_model() == plan.cost_model()
    step = lfa().GraphStep(plan, Wt, 8)
    for rep in range(2):
        step.replay().synchronize()
        assert plan.info_status(step.info) == 0
        vals, idx = to_np(step.vals), to_np(step.idx)
        for li, l in enumerate(layers):
            W64 = Ws[li].astype(np.float64)
            p, q, j = idx[li].T
            s_at = oracle.lfa_svd(W64, l.n, l.m, freqs=np.stack([p, q], axis=1))[np.arange(8), j]
            assert np.max(np.abs(vals[li] - s_at)) <= 1e-5 * s_at.max(), (rep, li)
            _grad_check(W64, l, idx[li], np.ones(8), step.dW[li], f"tuned graph {rep} layer {li}")
            if rep == 0:
                fr = _sample(l.n, l.m, 4, 60 + li)
                S_ref = oracle.lfa_svd(W64, l.n, l.m, freqs=fr)
                assert oracle.sigma_error(to_np(step.S[li])[fr[:, 0], fr[:, 1]], S_ref) <= 1e-5
    # the per-layer path of the tuned plan as well
    S, U, _, info = plan.svd(Wt)
    torch.cuda.synchronize()
    assert plan.info_status(info) == 0
    for li, l in enumerate(layers):
        fr = _sample(l.n, l.m, 4, 80 + li)
        S_ref = oracle.lfa_svd(Ws[li].astype(np.float64), l.n, l.m, freqs=fr)
        assert oracle.sigma_error(to_np(S[li])[fr[:, 0], fr[:, 1]], S_ref) <= 1e-5


@pytest.mark.parametrize("asm", [None, "bf16x2", "bf16x3"])
def test_large_grid_7x7_full_size_sampled(asm):
    """64 -> 64 channels, 7x7 kernel with five taps scaled by 1e3, 224x224
    grid (50176 symbols), sigma only, in each precision mode of the
    benchmark: 24 sampled symbols against the oracle within 1e-5 (the
    measured errors are 9e-7 FP32, 2e-6 bf16x2, 9e-7 bf16x3)."""
    banner(f"7x7 224x224 full size, asm={asm}")
    L, W, _ = workloads.large_grid_7x7()
    S, info = lfa().svd(_w(W), L.n, L.m, asm=asm, return_info=True)
    torch.cuda.synchronize()
    assert info[0] == 0 and info[3] == 0, info
    fr = _sample(L.n, L.m, 24, 7)
    S_ref = oracle.lfa_svd(W.astype(np.float64), L.n, L.m, freqs=fr)
    assert oracle.sigma_error(to_np(S)[fr[:, 0], fr[:, 1]], S_ref) <= 1e-5
    # the whole grid: Parseval, sum of sigma^2 = n m ||W||_F^2
    ss = torch.sum(S.double() ** 2).item()
    assert abs(ss / (L.n * L.m * np.sum(W.astype(np.float64) ** 2)) - 1) <= 1e-5


def test_sigma_sum_convenience_matches_topk_and_gradient():
    """sigma_sum (cached plan, scalar penalty) equals the sum of sigma_topk's
    values, and its gradient equals the oracle's gradient of the same sum."""
    banner("sigma_sum")
    layers, Ws = _small_stack(seed=17)
    layers, Ws = layers[:3], Ws[:3]
    Wt = [_w(W).requires_grad_(True) for W in Ws]
    total = lfa().sigma_sum(Wt, [(l.n, l.m) for l in layers], k=8)
    total.backward()
    torch.cuda.synchronize()
    ref_total = 0.0
    for li, l in enumerate(layers):
        s = oracle.lfa_svd(Ws[li].astype(np.float64), l.n, l.m)
        vals, picks = oracle.topk(s, 8)
        ref_total += float(vals.sum())
        _grad_check(Ws[li].astype(np.float64), l, picks, np.ones(8), Wt[li].grad, f"sigma_sum layer {li}")
    assert abs(float(total.detach()) - ref_total) <= 1e-5 * ref_total
