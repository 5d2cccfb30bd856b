"""Helpers shared by the GPU parity tests (comparison metrics, case banners).
No method arithmetic: expected values always come from ``oracle``."""

import sys

import numpy as np
import torch

EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53


def banner(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().cpu().numpy()


def sigma_gate(dtype):
    """sigma error gates: normwise per symbol, 1e-5 in FP32, 1e-12 in FP64."""
    return 1e-5 if dtype == torch.float32 else 1e-12


def ortho_gate(M, dtype):
    """Loss of orthogonality allowed for U and V columns: twice the Jacobi
    stopping threshold (2 sqrt(M) u, relative), plus the rounding of the
    accumulated rotations (a few hundred rotations per column, u each)."""
    eps = EPS32 if dtype == torch.float32 else EPS64
    return 4 * np.sqrt(max(M, 16)) * eps + 64 * eps * np.sqrt(M)


def resid_gate(M, dtype):
    """||A V - U S||_F / ||A||_F: rounding of the rotations applied to G and V
    (about u per rotation, a few hundred per column)."""
    eps = EPS32 if dtype == torch.float32 else EPS64
    return 64 * eps * np.sqrt(M) + 4 * np.sqrt(max(M, 16)) * eps


def check_vectors(A, S, U, V, dtype, tag=""):
    """A [..., c_out, c_in] (oracle, complex128); S, U, V from the GPU (numpy).
    Checks residual ||A V - U S||_F / ||A||_F, orthonormality of U and V."""
    c_out, c_in = A.shape[-2:]
    M = max(c_out, c_in)
    Sd = S.astype(np.float64)
    Ud = U.astype(np.complex128)
    Vd = V.astype(np.complex128)
    res = A @ Vd - Ud * Sd[..., None, :]
    nA = np.sqrt(np.sum(np.abs(A) ** 2, axis=(-2, -1)))
    nA = np.where(nA > 0, nA, 1.0)
    rel = np.sqrt(np.sum(np.abs(res) ** 2, axis=(-2, -1))) / nA
    r = S.shape[-1]
    eye = np.eye(r)
    ou = np.max(np.abs(np.conj(np.swapaxes(Ud, -1, -2)) @ Ud - eye))
    ov = np.max(np.abs(np.conj(np.swapaxes(Vd, -1, -2)) @ Vd - eye))
    assert rel.max() <= resid_gate(M, dtype), f"{tag} residual {rel.max():.3e}"
    assert ou <= ortho_gate(M, dtype), f"{tag} U orthonormality {ou:.3e}"
    assert ov <= ortho_gate(M, dtype), f"{tag} V orthonormality {ov:.3e}"
    return rel.max(), ou, ov


def check_projectors(S_ref, U_ref, V_ref, U, V, dtype, tag=""):
    """Gauge-invariant comparison with the oracle: for singular values with a
    relative gap to their neighbours, u_j v_j^H must match."""
    eps = 1e-6 if dtype == torch.float32 else 1e-13
    r = S_ref.shape[-1]
    smax = S_ref[..., :1]
    gap = np.full(S_ref.shape, np.inf)
    if r > 1:
        d = np.abs(np.diff(S_ref, axis=-1))
        gap[..., :-1] = np.minimum(gap[..., :-1], d)
        gap[..., 1:] = np.minimum(gap[..., 1:], d)
    rel_gap = gap / np.where(smax > 0, smax, 1.0)
    Ud, Vd = U.astype(np.complex128), V.astype(np.complex128)
    worst = 0.0
    flat_ok = rel_gap > 1e-3
    idx = np.argwhere(flat_ok)
    for ind in idx[:: max(1, len(idx) // 400)]:
        *lead, j = ind
        lead = tuple(lead)
        P_ref = np.outer(U_ref[lead][:, j], np.conj(V_ref[lead][:, j]))
        P = np.outer(Ud[lead][:, j], np.conj(Vd[lead][:, j]))
        err = np.max(np.abs(P - P_ref))
        bound = eps * (10 + 1.0 / rel_gap[lead + (j,)])
        worst = max(worst, err / bound)
        assert err <= bound, f"{tag} projector {lead}, j={j}: {err:.3e} > {bound:.3e}"
    return worst


def pick_gaps(S_sym, picks, grad=None):
    """Relative gap of each picked singular value: the distance from
    sigma_j(k) to the other singular values of the same symbol, over
    sigma_max(k), leaving out values picked in that symbol with the same
    weight (the gradient of a sum over a whole cluster of one symbol is
    well-posed; only a cut through a cluster makes the picked terms
    ill-conditioned).  ``S_sym [k, r]`` are the oracle's values of each
    pick's symbol, ``picks [k, 3]`` the (p, q, j), ``grad [k]`` the weights."""
    picks = np.asarray(picks)
    g = np.ones(len(picks)) if grad is None else np.asarray(grad, dtype=np.float64)
    gaps = np.empty(len(picks))
    for s, (p, q, j) in enumerate(picks):
        same = {int(picks[t, 2]) for t in range(len(picks))
                if picks[t, 0] == p and picks[t, 1] == q and g[t] == g[s]}
        sv = S_sym[s]
        d = [abs(sv[j] - sv[jj]) for jj in range(len(sv)) if jj not in same]
        gaps[s] = (min(d) if d else np.inf) / max(sv[0], np.finfo(np.float64).tiny)
    return gaps


GRAD_GATE = 1e-3          # dL/dW agreement with the oracle (relative)
GRAD_GAP_MIN = 1e-3       # picks separated by at least this relative gap


def grad_errors(dW, ref, S_sym, picks, grad=None, tag=""):
    """Gradient of a sum of picked singular values against the oracle's.

    The gate is elementwise: max |dW - ref| / max |ref| <= 1e-3, for picks
    whose singular values are separated from the rest of their symbol by a
    relative gap of at least 1e-3 (their singular vectors, and so each term
    of the gradient, are then determined to about u / gap).  When a pick sits
    in a tighter cluster, its singular vectors are ill-conditioned and only
    the Frobenius-relative error is gated (at the same 1e-3).  Returns
    (elementwise, frobenius, min gap)."""
    dW = np.asarray(dW, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    elem = float(np.max(np.abs(dW - ref)) / np.max(np.abs(ref)))
    frob = float(np.linalg.norm(dW - ref) / np.linalg.norm(ref))
    gap = float(np.min(pick_gaps(S_sym, picks, grad)))
    if gap >= GRAD_GAP_MIN:
        assert elem <= GRAD_GATE, f"{tag} gradient elementwise {elem:.3e} (gap {gap:.2e})"
    else:
        assert frob <= GRAD_GATE, f"{tag} gradient Frobenius {frob:.3e} (gap {gap:.2e} below 1e-3)"
    print(f"[grad] {tag} elementwise {elem:.2e} frobenius {frob:.2e} min gap {gap:.2e}", flush=True)
    return elem, frob, gap
