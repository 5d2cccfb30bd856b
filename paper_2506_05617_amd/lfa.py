"""PyTorch binding of liblfa: argument marshalling only.

Every step of the computation runs in the HIP kernels of liblfa.so; this
module checks shapes and dtypes, allocates outputs and workspace with torch
(device memory is owned by PyTorch's allocator) and passes raw pointers and
the current HIP stream through the C ABI.

Layouts (see include/lfa.h): W is [c_out, c_in, kh, kw]; symbols are
[n, m, c_out, c_in] complex; sigma is [n, m, r] (descending); U is
[n, m, c_out, r], V is [n, m, c_in, r] with A = U diag(sigma) V^H.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Sequence

import torch

from . import _lib
from ._lib import check, ptr_array


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(dtype):
    if dtype == torch.float32:
        return _lib.LFA_F32
    if dtype == torch.float64:
        return _lib.LFA_F64
    raise TypeError(f"weights must be float32 or float64, got {dtype}")


def _complex_of(dtype):
    return torch.complex64 if dtype == torch.float32 else torch.complex128


def _asm_flag(asm):
    return {None: 0, "valu": 0, "mfma": _lib.LFA_ASM_MFMA,
            "bf16x2": _lib.LFA_ASM_BF16X2, "bf16x3": _lib.LFA_ASM_BF16X3}[asm]


@dataclass(frozen=True)
class LayerSpec:
    c_out: int
    c_in: int
    kh: int
    kw: int
    n: int
    m: int

    @property
    def r(self):
        return min(self.c_out, self.c_in)


class Plan:
    """An lfa_plan: layer shapes, dtype and flags fixed at creation.

    Workspace is allocated lazily on the device of the first call and reused.
    """

    def __init__(self, layers: Sequence[LayerSpec], dtype=torch.float32, want_u=False,
                 want_v=False, asm=None, phase_normalize=False):
        self.lib = _lib.load()
        self.layers = [LayerSpec(*l) if not isinstance(l, LayerSpec) else l for l in layers]
        self.dtype = dtype
        self.want_u, self.want_v, self.asm = want_u, want_v, asm
        flags = (_lib.LFA_WANT_U if want_u else 0) | (_lib.LFA_WANT_V if want_v else 0) | _asm_flag(asm)
        if phase_normalize:
            flags |= _lib.LFA_PHASE_NORMALIZE
        arr = (_lib.LfaLayer * len(self.layers))(
            *[_lib.LfaLayer(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in self.layers])
        h = ctypes.c_void_p()
        check(self.lib.lfa_plan_create(ctypes.byref(h), arr, len(self.layers),
                                       _dtype_code(dtype), flags), "lfa_plan_create")
        self.handle = h
        nb = ctypes.c_size_t()
        check(self.lib.lfa_plan_workspace_bytes(h, ctypes.byref(nb)), "lfa_plan_workspace_bytes")
        self.ws_bytes = nb.value
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.lfa_plan_destroy(h)
            self.handle = None

    def prepare(self, k=0):
        """Upload the plan's device tables to the current device (and the
        persistent gradient's work list for k > 0) ahead of graph capture
        (lfa_plan_prepare)."""
        check(self.lib.lfa_plan_prepare(self.handle, int(k)), "lfa_plan_prepare")

    def record_phases(self, ticks):
        """Phase record of the register kernel (lfa_plan_record_phases):
        `ticks` a cleared int64 CUDA tensor of 4 (load, sweeps, finish, save;
        100 MHz ticks summed over the groups) that later svd() calls add to,
        or None to stop.  The plan keeps a reference until then."""
        if ticks is not None and (ticks.dtype != torch.int64 or ticks.numel() < 4 or not ticks.is_cuda
                                  or not ticks.is_contiguous()):
            raise ValueError("ticks must be a contiguous int64 CUDA tensor of 4")
        self._phase_ticks = ticks
        check(self.lib.lfa_plan_record_phases(self.handle, None if ticks is None else
                                              ctypes.c_void_p(ticks.data_ptr())), "lfa_plan_record_phases")

    def set_max_sweeps(self, max_sweeps):
        """Cap on Jacobi sweeps per symbol (1 .. 40) for later calls."""
        check(self.lib.lfa_plan_set_max_sweeps(self.handle, int(max_sweeps)), "lfa_plan_set_max_sweeps")

    def info_status(self, info):
        """Warnings of a finished call from its info record [L, LFA_INFO_WORDS]: 0, or the
        OR of LFA_WARN_NOT_CONVERGED / _NONFINITE / _TEAM_TIMEOUT
        (lfa_info_status)."""
        host = info.detach().to("cpu", torch.int32).contiguous()
        return check(self.lib.lfa_info_status(ctypes.cast(host.data_ptr(), _lib.I32P), host.shape[0]),
                     "lfa_info_status")

    def workspace(self, device):
        if self._ws is None or self._ws.device != device:
            self._ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)
        return self._ws

    def queue_info(self, layer):
        """(resident work-groups, sweeps per turn) of the layer's work-queue
        launch on the current device; (0, ...) when it has none."""
        vals = [ctypes.c_int32() for _ in range(2)]
        check(self.lib.lfa_plan_queue_info(self.handle, layer, *[ctypes.byref(v) for v in vals]),
              "lfa_plan_queue_info")
        return tuple(v.value for v in vals)

    def preconditioned(self, layer):
        """True when svd() runs the layer through QR preconditioning."""
        v = ctypes.c_int32()
        check(self.lib.lfa_plan_preconditioned(self.handle, layer, ctypes.byref(v)), "lfa_plan_preconditioned")
        return bool(v.value)

    def launch_shape(self, layer):
        vals = [ctypes.c_int32() for _ in range(4)]
        check(self.lib.lfa_plan_launch_shape(self.handle, layer, *[ctypes.byref(v) for v in vals]),
              "lfa_plan_launch_shape")
        return tuple(v.value for v in vals)

    # -- checks --------------------------------------------------------------
    def _check_weights(self, Ws):
        if len(Ws) != len(self.layers):
            raise ValueError("one weight tensor per layer")
        dev = Ws[0].device
        for W, l in zip(Ws, self.layers):
            if W.device.type != "cuda":
                raise ValueError("weights must be on the GPU")
            if W.device != dev:
                raise ValueError("all weights on one device")
            if W.dtype != self.dtype:
                raise TypeError(f"weights must be {self.dtype}")
            if tuple(W.shape) != (l.c_out, l.c_in, l.kh, l.kw) or not W.is_contiguous():
                raise ValueError(f"weight of shape {tuple(W.shape)} does not match {l}")
        return dev

    def _alloc_outputs(self, dev, want_u, want_v, count=None):
        cdt = _complex_of(self.dtype)
        S, U, V = [], [], []
        for l in self.layers:
            lead = (l.n, l.m) if count is None else (count,)
            S.append(torch.empty(*lead, l.r, dtype=self.dtype, device=dev))
            U.append(torch.empty(*lead, l.c_out, l.r, dtype=cdt, device=dev) if want_u else None)
            V.append(torch.empty(*lead, l.c_in, l.r, dtype=cdt, device=dev) if want_v else None)
        return S, U, V

    # -- entry points -------------------------------------------------------
    def symbols(self, Ws):
        dev = self._check_weights(Ws)
        cdt = _complex_of(self.dtype)
        A = [torch.empty(l.n, l.m, l.c_out, l.c_in, dtype=cdt, device=dev) for l in self.layers]
        w, _k1 = ptr_array([W.data_ptr() for W in Ws])
        a, _k2 = ptr_array([x.data_ptr() for x in A])
        check(self.lib.lfa_symbols(self.handle, w, a, _stream_ptr()), "lfa_symbols")
        return A

    def _info(self, info, dev):
        """The caller's info record, checked (the library writes
        LFA_INFO_WORDS int32 per layer into it), or a new one."""
        if info is None:
            return torch.zeros(len(self.layers), _lib.LFA_INFO_WORDS, dtype=torch.int32, device=dev)
        if (info.dtype != torch.int32 or tuple(info.shape) != (len(self.layers), _lib.LFA_INFO_WORDS)
                or not info.is_contiguous() or info.device != dev):
            raise ValueError(f"info must be a contiguous int32 tensor [{len(self.layers)}, "
                             f"{_lib.LFA_INFO_WORDS}] on {dev}, got {tuple(info.shape)} {info.dtype} "
                             f"on {info.device}")
        return info

    def _svd_call(self, fn, name, inputs, dev, info=None, out=None):
        S, U, V = out if out is not None else self._alloc_outputs(dev, self.want_u, self.want_v)
        info = self._info(info, dev)
        ws = self.workspace(dev)
        i_arr, _k0 = ptr_array([x.data_ptr() for x in inputs])
        s_arr, _k1 = ptr_array([x.data_ptr() for x in S])
        u_arr, _k2 = ptr_array([x.data_ptr() if x is not None else 0 for x in U])
        v_arr, _k3 = ptr_array([x.data_ptr() if x is not None else 0 for x in V])
        check(fn(self.handle, i_arr, s_arr, u_arr if self.want_u else None,
                 v_arr if self.want_v else None, ctypes.c_void_p(info.data_ptr()),
                 ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), _stream_ptr()), name)
        return S, U, V, info

    def svd(self, Ws, persistent=False, info=None, out=None):
        """SVD of every symbol of every layer.  Returns lists (S, U, V, info)."""
        dev = self._check_weights(Ws)
        fn = self.lib.lfa_svd_persistent if persistent else self.lib.lfa_svd
        return self._svd_call(fn, "lfa_svd_persistent" if persistent else "lfa_svd", Ws, dev, info, out)

    def svd_noalloc(self, Ws, info=None, out=None):
        """As svd(), through lfa_svd_noalloc: no workspace, the library's static
        device scratch instead (outputs are still the caller's: allocated
        here with torch unless `out` is given).  Returns (S, U, V, info)."""
        dev = self._check_weights(Ws)
        S, U, V = out if out is not None else self._alloc_outputs(dev, self.want_u, self.want_v)
        info = self._info(info, dev)
        w_arr, _k0 = ptr_array([x.data_ptr() for x in Ws])
        s_arr, _k1 = ptr_array([x.data_ptr() for x in S])
        u_arr, _k2 = ptr_array([x.data_ptr() if x is not None else 0 for x in U])
        v_arr, _k3 = ptr_array([x.data_ptr() if x is not None else 0 for x in V])
        check(self.lib.lfa_svd_noalloc(self.handle, w_arr, s_arr, u_arr if self.want_u else None,
                                       v_arr if self.want_v else None, ctypes.c_void_p(info.data_ptr()),
                                       _stream_ptr()), "lfa_svd_noalloc")
        return S, U, V, info

    def persistent_busy(self, Ws, out=None):
        """One lfa_svd_persistent_busy launch: (S, U, V, info, records) with
        records an int64 [grid, 4] tensor (busy ticks at 100 MHz, items, XCD,
        HW_ID compute-unit bits) per work-group."""
        dev = self._check_weights(Ws)
        g = ctypes.c_int32()
        check(self.lib.lfa_plan_persistent_grid(self.handle, ctypes.byref(g)), "lfa_plan_persistent_grid")
        S, U, V = out if out is not None else self._alloc_outputs(dev, self.want_u, self.want_v)
        info = torch.zeros(len(self.layers), _lib.LFA_INFO_WORDS, dtype=torch.int32, device=dev)
        rec = torch.zeros(max(1, g.value), 4, dtype=torch.int64, device=dev)
        ws = self.workspace(dev)
        w_arr, _k0 = ptr_array([x.data_ptr() for x in Ws])
        s_arr, _k1 = ptr_array([x.data_ptr() for x in S])
        u_arr, _k2 = ptr_array([x.data_ptr() if x is not None else 0 for x in U])
        v_arr, _k3 = ptr_array([x.data_ptr() if x is not None else 0 for x in V])
        check(self.lib.lfa_svd_persistent_busy(self.handle, w_arr, s_arr, u_arr if self.want_u else None,
                                               v_arr if self.want_v else None, ctypes.c_void_p(info.data_ptr()),
                                               ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                               ctypes.c_void_p(rec.data_ptr()), rec.shape[0], _stream_ptr()),
              "lfa_svd_persistent_busy")
        return S, U, V, info, rec

    def svd_symbols(self, As, info=None):
        cdt = _complex_of(self.dtype)
        for A, l in zip(As, self.layers):
            if A.dtype != cdt or tuple(A.shape) != (l.n, l.m, l.c_out, l.c_in) or not A.is_contiguous():
                raise ValueError("symbols must be contiguous [n, m, c_out, c_in] complex")
        return self._svd_call(self.lib.lfa_svd_symbols, "lfa_svd_symbols", As, As[0].device, info)

    def apply(self, layer, S, U, V, x, kind="identity", param=0.0):
        """Spectral function of layer `layer`'s operator applied to images
        ``x [batch, c_x, n, m]`` through its SVD ``S, U, V`` (as ``svd``
        returns them for that layer, with U and V): ``identity`` (the
        convolution), ``clip`` (singular values clipped at ``param``),
        ``truncate`` (singular values at or below ``param`` dropped: a
        low-rank truncation) or ``pinv`` (pseudo-inverse with absolute
        cut-off ``param``; x has c_out channels and y has c_in).  Returns
        ``y [batch, c_y, n, m]``."""
        kinds = {"identity": _lib.LFA_SPECTRAL_IDENTITY, "clip": _lib.LFA_SPECTRAL_CLIP,
                 "pinv": _lib.LFA_SPECTRAL_PINV, "truncate": _lib.LFA_SPECTRAL_TRUNCATE}
        l = self.layers[layer]
        cx, cy = (l.c_out, l.c_in) if kind == "pinv" else (l.c_in, l.c_out)
        if x.dtype != self.dtype or x.dim() != 4 or tuple(x.shape[1:]) != (cx, l.n, l.m) or not x.is_contiguous():
            raise ValueError(f"x must be contiguous [batch, {cx}, {l.n}, {l.m}] {self.dtype}")
        cdt = _complex_of(self.dtype)
        r = l.r
        if tuple(S.shape) != (l.n, l.m, r) or tuple(U.shape) != (l.n, l.m, l.c_out, r) or \
                tuple(V.shape) != (l.n, l.m, l.c_in, r) or U.dtype != cdt or V.dtype != cdt or S.dtype != self.dtype:
            raise ValueError("S, U, V must be this layer's SVD")
        batch = x.shape[0]
        y = torch.empty(batch, cy, l.n, l.m, dtype=self.dtype, device=x.device)
        nbytes = ctypes.c_size_t()
        check(self.lib.lfa_apply_workspace_bytes(self.handle, layer, batch, ctypes.byref(nbytes)),
              "lfa_apply_workspace_bytes")
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=x.device)
        check(self.lib.lfa_apply(self.handle, layer, ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(V.data_ptr()), kinds[kind], float(param),
                                 ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), batch,
                                 ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), _stream_ptr()),
              "lfa_apply")
        return y

    def lift(self, layer, U, V, idx):
        """Global singular vectors of layer `layer` for picks ``idx [count, 3]``
        (int32 (p, q, j) on the device): ``(u_hat [count, c_out, n, m],
        v_hat [count, c_in, n, m])`` complex, the Fourier mode of (p, q) times
        column j of U and V at (p, q), unit norm.  U or V may be None (that
        output is then None)."""
        l = self.layers[layer]
        cdt = _complex_of(self.dtype)
        for T, c in ((U, l.c_out), (V, l.c_in)):
            if T is not None and (tuple(T.shape) != (l.n, l.m, c, l.r) or T.dtype != cdt or not T.is_contiguous()):
                raise ValueError("U, V must be this layer's singular vectors")
        if idx.dtype != torch.int32 or idx.dim() != 2 or idx.shape[1] != 3 or not idx.is_contiguous():
            raise ValueError("idx must be contiguous int32 [count, 3]")
        count = idx.shape[0]
        dev = idx.device
        uh = None if U is None else torch.empty(count, l.c_out, l.n, l.m, dtype=cdt, device=dev)
        vh = None if V is None else torch.empty(count, l.c_in, l.n, l.m, dtype=cdt, device=dev)
        ptr = lambda t: ctypes.c_void_p(None if t is None else t.data_ptr())
        check(self.lib.lfa_lift(self.handle, layer, ptr(U), ptr(V), ptr(idx), count, ptr(uh), ptr(vh),
                                _stream_ptr()), "lfa_lift")
        return uh, vh

    def topk(self, S, k):
        dev = S[0].device
        vals = torch.empty(len(self.layers), k, dtype=self.dtype, device=dev)
        idx = torch.empty(len(self.layers), k, 3, dtype=torch.int32, device=dev)
        s_arr, _k = ptr_array([x.data_ptr() for x in S])
        check(self.lib.lfa_topk(self.handle, s_arr, k, ctypes.c_void_p(vals.data_ptr()),
                                ctypes.c_void_p(idx.data_ptr()), _stream_ptr()), "lfa_topk")
        return vals, idx

    def adjoint(self, U, V, idx, grad):
        dev = idx.device
        k = idx.shape[1]
        dW = [torch.empty(l.c_out, l.c_in, l.kh, l.kw, dtype=self.dtype, device=dev) for l in self.layers]
        u_arr, _k1 = ptr_array([x.data_ptr() for x in U])
        v_arr, _k2 = ptr_array([x.data_ptr() for x in V])
        d_arr, _k3 = ptr_array([x.data_ptr() for x in dW])
        idx = idx.contiguous()
        grad = grad.to(self.dtype).contiguous()
        check(self.lib.lfa_adjoint(self.handle, u_arr, v_arr, ctypes.c_void_p(idx.data_ptr()),
                                   ctypes.c_void_p(grad.data_ptr()), k, d_arr, _stream_ptr()),
              "lfa_adjoint")
        return dW

    def adjoint_onesided(self, Ws, S, X, idx, grad, out=None):
        """dW of sum_s g_s sigma_s from the kept side X of each layer's SVD
        (U for c_out >= c_in, V otherwise; as svd() writes it) and the
        weights, which give the other side of each pick (lfa_adjoint_onesided)."""
        dev = self._check_weights(Ws)
        k = idx.shape[1]
        dW = out if out is not None else [
            torch.empty(l.c_out, l.c_in, l.kh, l.kw, dtype=self.dtype, device=dev) for l in self.layers]
        ws = self.workspace(dev)
        w_arr, _k0 = ptr_array([x.data_ptr() for x in Ws])
        s_arr, _k1 = ptr_array([x.data_ptr() for x in S])
        x_arr, _k2 = ptr_array([x.data_ptr() for x in X])
        d_arr, _k3 = ptr_array([x.data_ptr() for x in dW])
        idx = idx.contiguous()
        grad = grad.to(self.dtype).contiguous()
        check(self.lib.lfa_adjoint_onesided(self.handle, w_arr, s_arr, x_arr, ctypes.c_void_p(idx.data_ptr()),
                                            ctypes.c_void_p(grad.data_ptr()), k, d_arr,
                                            ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                            _stream_ptr()), "lfa_adjoint_onesided")
        return dW

    def sigma_grad(self, Ws, idx, grad, out=None, persistent=False):
        dev = self._check_weights(Ws)
        k = idx.shape[1]
        dW = out if out is not None else [
            torch.empty(l.c_out, l.c_in, l.kh, l.kw, dtype=self.dtype, device=dev) for l in self.layers]
        ws = self.workspace(dev)
        w_arr, _k1 = ptr_array([x.data_ptr() for x in Ws])
        d_arr, _k2 = ptr_array([x.data_ptr() for x in dW])
        idx = idx.contiguous()
        grad = grad.to(self.dtype).contiguous()
        fn = self.lib.lfa_sigma_grad_persistent if persistent else self.lib.lfa_sigma_grad
        check(fn(self.handle, w_arr, ctypes.c_void_p(idx.data_ptr()),
                 ctypes.c_void_p(grad.data_ptr()), k, d_arr,
                 ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                 _stream_ptr()), "lfa_sigma_grad_persistent" if persistent else "lfa_sigma_grad")
        return dW

    def autotune(self, Ws, cache_path=None, layers=True, persistent=True):
        """Time and choose the plan's launch parameters on these weights
        (lfa_autotune), with an optional JSON cache file.  The workspace size
        may change: the plan's cached workspace is dropped."""
        dev = self._check_weights(Ws)
        S, U, V = self._alloc_outputs(dev, self.want_u, self.want_v)
        w_arr, _k0 = ptr_array([x.data_ptr() for x in Ws])
        s_arr, _k1 = ptr_array([x.data_ptr() for x in S])
        u_arr, _k2 = ptr_array([x.data_ptr() if x is not None else 0 for x in U])
        v_arr, _k3 = ptr_array([x.data_ptr() if x is not None else 0 for x in V])
        what = (_lib.LFA_TUNE_LAYERS if layers else 0) | (_lib.LFA_TUNE_PERSISTENT if persistent else 0)
        torch.cuda.current_stream().synchronize()
        check(self.lib.lfa_autotune(self.handle, w_arr, s_arr, u_arr if self.want_u else None,
                                    v_arr if self.want_v else None,
                                    None if cache_path is None else str(cache_path).encode(), what,
                                    _stream_ptr()), "lfa_autotune")
        nb = ctypes.c_size_t()
        check(self.lib.lfa_plan_workspace_bytes(self.handle, ctypes.byref(nb)), "lfa_plan_workspace_bytes")
        self.ws_bytes = nb.value
        self._ws = None

    def tuning(self, layer):
        """(qr, queue_seg, team_w, asm_mat) chosen for a layer."""
        vals = [ctypes.c_int32() for _ in range(4)]
        check(self.lib.lfa_plan_tuning(self.handle, layer, *[ctypes.byref(v) for v in vals]), "lfa_plan_tuning")
        return tuple(v.value for v in vals)

    def cost_model(self):
        """(seconds per unit of a register-kernel wave, of a blocked work-group, team overhead)."""
        vals = [ctypes.c_double() for _ in range(3)]
        check(self.lib.lfa_plan_cost_model(self.handle, *[ctypes.byref(v) for v in vals]), "lfa_plan_cost_model")
        return tuple(v.value for v in vals)


class GraphStep:
    """HIP graph of [persistent SVD -> top-k -> sigma gradient] for fixed
    buffers.  Copy new weights into ``self.W`` and call ``replay()``.

    With a sigma-only plan the gradient recomputes the singular vectors of the
    picked symbols (lfa_graph_create).  With a plan that wants U and V the
    forward pass keeps them for every symbol (``self.U``, ``self.V``) and the
    gradient is one adjoint launch (lfa_graph_create_uv).  With a plan that
    wants only U (every layer c_out >= c_in) or only V (every layer
    c_out < c_in) the forward pass keeps that side, which needs no rotation
    accumulator, and the gradient recomputes the other side of each pick
    from the weights (lfa_graph_create_onesided)."""

    def __init__(self, plan: Plan, Ws, k, grad=None, stream=None):
        self.plan = plan
        dev = plan._check_weights(Ws)
        self.W = Ws
        self.k = k
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        uv = plan.want_u and plan.want_v
        one = plan.want_u != plan.want_v
        self.S, self.U, self.V = plan._alloc_outputs(dev, plan.want_u, plan.want_v)
        L = len(plan.layers)
        self.vals = torch.empty(L, k, dtype=plan.dtype, device=dev)
        self.idx = torch.empty(L, k, 3, dtype=torch.int32, device=dev)
        self.grad = (torch.ones(L, k, dtype=plan.dtype, device=dev) if grad is None
                     else grad.to(plan.dtype).contiguous())
        self.dW = [torch.empty_like(W) for W in Ws]
        self.info = torch.zeros(L, _lib.LFA_INFO_WORDS, dtype=torch.int32, device=dev)
        # a workspace of its own: replays run on self.stream and must not
        # share counters and slots with eager calls on the plan
        ws = torch.empty(max(plan.ws_bytes, 256), dtype=torch.uint8, device=dev)
        self._done = torch.cuda.Event()
        self._keep = []
        w_arr, k0 = ptr_array([x.data_ptr() for x in Ws])
        s_arr, k1 = ptr_array([x.data_ptr() for x in self.S])
        d_arr, k2 = ptr_array([x.data_ptr() for x in self.dW])
        self._keep += [k0, k1, k2, ws]
        h = ctypes.c_void_p()
        torch.cuda.synchronize(dev)
        tail = (k, ctypes.c_void_p(self.vals.data_ptr()), ctypes.c_void_p(self.idx.data_ptr()),
                ctypes.c_void_p(self.grad.data_ptr()), d_arr, ctypes.c_void_p(self.info.data_ptr()),
                ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if uv:
            u_arr, k3 = ptr_array([x.data_ptr() for x in self.U])
            v_arr, k4 = ptr_array([x.data_ptr() for x in self.V])
            self._keep += [k3, k4]
            check(plan.lib.lfa_graph_create_uv(plan.handle, w_arr, s_arr, u_arr, v_arr, *tail),
                  "lfa_graph_create_uv")
        elif one:
            self.X = self.U if plan.want_u else self.V
            x_arr, k3 = ptr_array([x.data_ptr() for x in self.X])
            self._keep += [k3]
            check(plan.lib.lfa_graph_create_onesided(plan.handle, w_arr, s_arr, x_arr, *tail),
                  "lfa_graph_create_onesided")
        else:
            check(plan.lib.lfa_graph_create(plan.handle, w_arr, s_arr, *tail), "lfa_graph_create")
        self.handle = h

    def replay(self):
        """Launch the graph on self.stream after the work queued so far on the
        current stream (new weights, reads of the last replay's outputs), and
        make the current stream wait for it.  Returns self.stream."""
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        check(self.plan.lib.lfa_graph_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)),
              "lfa_graph_launch")
        self._done.record(self.stream)
        cur.wait_event(self._done)
        return self.stream

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.plan.lib.lfa_graph_destroy(h)
            self.handle = None


# ---------------------------------------------------------------------------
# Convenience functions
# ---------------------------------------------------------------------------

_PLANS = {}


def _plan_for(specs, dtype, want_u, want_v, asm=None, phase_normalize=False):
    key = (tuple(specs), dtype, want_u, want_v, asm, phase_normalize)
    p = _PLANS.get(key)
    if p is None:
        p = Plan(specs, dtype, want_u, want_v, asm, phase_normalize)
        _PLANS[key] = p
    return p


def _spec(W, n, m):
    c_out, c_in, kh, kw = W.shape
    return LayerSpec(c_out, c_in, kh, kw, n, n if m is None else m)


def symbols(W, n, m=None, asm=None):
    """Symbols [n, m, c_out, c_in] of one layer (lfa_symbols)."""
    return _plan_for([_spec(W, n, m)], W.dtype, False, False, asm).symbols([W])[0]


def svd(W, n, m=None, compute_uv=False, asm=None, return_info=False, phase_normalize=False):
    """Singular values [n, m, r] (and U, V if compute_uv) of one layer; with
    phase_normalize (and compute_uv) every pair (u_j, v_j) is multiplied by
    the phase that makes the largest-modulus entry of v_j real positive."""
    p = _plan_for([_spec(W, n, m)], W.dtype, compute_uv, compute_uv, asm, phase_normalize and compute_uv)
    S, U, V, info = p.svd([W])
    out = (S[0], U[0], V[0]) if compute_uv else S[0]
    return (out, info[0]) if return_info else out


def crystal_layer(spec: LayerSpec, stride: int) -> LayerSpec:
    """The stride-1 layer on the coarse torus of a stride-`stride` layer read
    as a crystal (lfa_crystal_layer): (c_out, s*s*c_in, kh', kw', n/s, m/s)."""
    lib = _lib.load()
    out = _lib.LfaLayer()
    src = _lib.LfaLayer(spec.c_out, spec.c_in, spec.kh, spec.kw, spec.n, spec.m)
    check(lib.lfa_crystal_layer(ctypes.byref(src), stride, ctypes.byref(out)), "lfa_crystal_layer")
    return LayerSpec(out.c_out, out.c_in, out.kh, out.kw, out.n, out.m)


def crystal_weights(W, spec: LayerSpec, stride: int, adjoint=False):
    """Weights of the crystal form of a stride-`stride` layer (lfa_crystal_weights):
    ``W [c_out, c_in, kh, kw] -> Wc [c_out, s*s*c_in, kh', kw']``, or with
    ``adjoint`` the transpose ``Wc -> W`` (for gradients)."""
    lib = _lib.load()
    c = crystal_layer(spec, stride)
    shape_in, shape_out = (spec.c_out, spec.c_in, spec.kh, spec.kw), (c.c_out, c.c_in, c.kh, c.kw)
    if adjoint:
        shape_in, shape_out = shape_out, shape_in
    if tuple(W.shape) != shape_in or not W.is_contiguous() or W.device.type != "cuda":
        raise ValueError(f"expected a contiguous GPU tensor of shape {shape_in}")
    out = torch.empty(shape_out, dtype=W.dtype, device=W.device)
    src = _lib.LfaLayer(spec.c_out, spec.c_in, spec.kh, spec.kw, spec.n, spec.m)
    check(lib.lfa_crystal_weights(ctypes.byref(src), stride, _dtype_code(W.dtype), ctypes.c_void_p(W.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()),
                                  _lib.LFA_CRYSTAL_ADJOINT if adjoint else _lib.LFA_CRYSTAL_FORWARD,
                                  _stream_ptr()), "lfa_crystal_weights")
    return out


class SigmaTopK(torch.autograd.Function):
    """Per-layer top-k singular values of a stack of periodic convolutions,
    differentiable in the weights: forward = one persistent sigma-only SVD
    launch + top-k; backward = SVD with vectors of the selected symbols +
    adjoint kernel (lfa_sigma_grad)."""

    @staticmethod
    def forward(ctx, plan: Plan, k: int, *Ws):
        S, _, _, info = plan.svd(list(Ws), persistent=True)
        vals, idx = plan.topk(S, k)
        ctx.plan = plan
        ctx.save_for_backward(idx, *Ws)
        ctx.mark_non_differentiable(idx)
        return vals, idx

    @staticmethod
    def backward(ctx, grad_vals, _grad_idx):
        idx, *Ws = ctx.saved_tensors
        dW = ctx.plan.sigma_grad(list(Ws), idx, grad_vals.contiguous(), persistent=True)
        return (None, None, *dW)


def sigma_topk(plan: Plan, Ws, k: int):
    """Differentiable per-layer top-k singular values: returns (vals [L, k], idx [L, k, 3])."""
    return SigmaTopK.apply(plan, k, *Ws)


def sigma_sum(Ws, grids, k: int = 8):
    """The sum over layers of each layer's k largest singular values, as a
    differentiable scalar (a spectral-norm style penalty): ``Ws`` are the
    layers' weights, ``grids`` their (n, m) grids (or n for square grids).
    The plan for these shapes is built on first use and cached."""
    grids = [(g, g) if isinstance(g, int) else tuple(g) for g in grids]
    specs = tuple(_spec(W, n, m) for W, (n, m) in zip(Ws, grids))
    plan = _plan_for(specs, Ws[0].dtype, False, False)
    vals, _ = SigmaTopK.apply(plan, k, *Ws)
    return vals.sum()
