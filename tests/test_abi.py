"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/lfa.h, and rejects bad plans at enqueue time."""

import ctypes
import os
import re

import pytest

import paper_2506_05617_amd as lfa
from paper_2506_05617_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lfa.h")

needs_lib = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                               reason="liblfa.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lfa_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for must in ["lfa_plan_create", "lfa_symbols", "lfa_svd", "lfa_svd_persistent", "lfa_topk",
                 "lfa_adjoint", "lfa_sigma_grad", "lfa_graph_create", "lfa_graph_create_uv", "lfa_autotune",
                 "lfa_status_string"]:
        assert must in names
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


@needs_lib
def test_status_strings_and_version():
    lib = lfa.load()
    assert lib.lfa_version() == 1
    for code in (0, -1, -2, -3, -4, -5, 12345):
        assert lib.lfa_status_string(code)
    assert lib.lfa_last_hip_error() == 0


def _create(layers, dtype=0, flags=0):
    lib = lfa.load()
    arr = (_lib.LfaLayer * len(layers))(*[_lib.LfaLayer(*l) for l in layers])
    h = ctypes.c_void_p()
    st = lib.lfa_plan_create(ctypes.byref(h), arr, len(layers), dtype, flags)
    if st == 0:
        lib.lfa_plan_destroy(h)
    else:
        assert not h.value
    return st


@needs_lib
@pytest.mark.parametrize("layer,dtype,flags,expect", [
    ((16, 16, 3, 3, 32, 32), 0, 0, 0),
    ((16, 16, 3, 3, 32, 32), 1, 3, 0),
    ((0, 16, 3, 3, 32, 32), 0, 0, -1),            # empty channel
    ((16, 16, 3, 3, 0, 32), 0, 0, -1),            # empty grid
    ((16, 16, 5, 5, 4, 4), 0, 0, -1),             # kernel wider than the grid
    ((16, 16, 3, 3, 32, 32), 2, 0, -1),           # unknown dtype
    ((16, 16, 3, 3, 32, 32), 0, 1 << 10, -1),     # unknown flag
    ((16, 16, 3, 3, 32, 32), 0, 8 | 16, -1),      # two assembly modes
    ((16, 16, 3, 3, 32, 32), 1, 8, -2),           # BF16 assembly needs FP32
    ((16, 16, 3, 3, 32, 32), 0, 32, -1),          # phase normalisation without vectors
    ((16, 16, 3, 3, 32, 32), 0, 32 | 2, 0),       # ... with V
    ((16, 16, 3, 3, 32, 32), 1, 32 | 1, 0),       # ... with U alone
    ((1024, 16, 3, 3, 8, 8), 0, 0, -2),           # more rows than one work-group holds
    ((16, 16, 13, 13, 16, 16), 0, 0, -2),         # more than 128 taps
])
def test_plan_validation(layer, dtype, flags, expect):
    assert _create([layer], dtype, flags) == expect


@needs_lib
def test_null_and_count_arguments():
    lib = lfa.load()
    h = ctypes.c_void_p()
    arr = (_lib.LfaLayer * 1)(_lib.LfaLayer(4, 4, 3, 3, 8, 8))
    assert lib.lfa_plan_create(None, arr, 1, 0, 0) == -1
    assert lib.lfa_plan_create(ctypes.byref(h), None, 1, 0, 0) == -1
    assert lib.lfa_plan_create(ctypes.byref(h), arr, 0, 0, 0) == -1
    assert lib.lfa_plan_destroy(None) == 0
    assert lib.lfa_svd(None, None, None, None, None, None, None, 0, None) == -1
    assert lib.lfa_topk(None, None, 8, None, None, None) == -1


@needs_lib
def test_compute_calls_reject_bad_arguments_before_touching_the_gpu():
    plan = lfa.Plan([lfa.LayerSpec(8, 8, 3, 3, 8, 8)])
    lib = plan.lib
    pp, keep = _lib.ptr_array([0])
    # null weight pointer in the per-layer array
    assert lib.lfa_svd(plan.handle, pp, pp, None, None, None, None, 0, None) == -1
    one, keep1 = _lib.ptr_array([1 << 20])
    # workspace missing
    assert lib.lfa_svd(plan.handle, one, one, None, None, None, None, 0, None) == -3
    # k out of range
    assert lib.lfa_topk(plan.handle, one, 0, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1
    assert lib.lfa_topk(plan.handle, one, 65, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1
    # graph forms: the vectors form needs U and V and a plan that wants both,
    # the sigma-only form a plan that wants neither
    h = ctypes.c_void_p()
    c1 = ctypes.c_void_p(1)
    uv = lfa.Plan([lfa.LayerSpec(8, 8, 3, 3, 8, 8)], want_u=True, want_v=True)
    assert lib.lfa_graph_create_uv(plan.handle, one, one, one, one, 8, c1, c1, c1, one, None, c1,
                                   1 << 30, c1, ctypes.byref(h)) == -2
    assert lib.lfa_graph_create_uv(uv.handle, one, one, None, one, 8, c1, c1, c1, one, None, c1,
                                   1 << 30, c1, ctypes.byref(h)) == -1
    assert lib.lfa_graph_create(uv.handle, one, one, 8, c1, c1, c1, one, None, c1, 1 << 30, c1,
                                ctypes.byref(h)) == -2
    assert h.value is None


@needs_lib
def test_workspace_and_launch_shapes():
    small = lfa.Plan([lfa.LayerSpec(16, 16, 3, 3, 32, 32)])
    L, threads, spg, storage = small.launch_shape(0)
    assert (L, storage) == (2, 0) and threads >= 64
    big = lfa.Plan([lfa.LayerSpec(512, 256, 3, 3, 32, 32)], want_u=True, want_v=True)
    L, threads, spg, storage = big.launch_shape(0)
    assert (threads, storage) == (512, 1)          # blocked kernel: one thread per row
    assert big.ws_bytes > 512 * 256 * 8
    wide = lfa.Plan([lfa.LayerSpec(3, 64, 3, 3, 8, 8)])     # c_out < c_in: works on A^H
    assert wide.launch_shape(0)[0] == 8


@needs_lib
def test_crystal_layer_shapes_and_errors():
    """lfa_crystal_layer (host only): the stride-1 layer of a strided layer's
    crystal form; the kernel extent covers the coarse tap offsets
    floor(y / s) of the centred taps y, which is checked here by listing
    them."""
    lib = lfa.load()

    def call(spec, s):
        out = _lib.LfaLayer()
        st = lib.lfa_crystal_layer(ctypes.byref(_lib.LfaLayer(*spec)), s, ctypes.byref(out))
        return st, (out.c_out, out.c_in, out.kh, out.kw, out.n, out.m)

    for spec, s in [((64, 64, 3, 3, 32, 32), 2), ((64, 3, 7, 7, 224, 224), 2), ((128, 64, 1, 1, 32, 32), 2),
                    ((8, 4, 4, 2, 12, 12), 3), ((8, 4, 3, 3, 10, 6), 1), ((8, 4, 5, 5, 20, 20), 4)]:
        st, got = call(spec, s)
        assert st == 0
        c_out, c_in, kh, kw, n, m = spec
        assert got[:2] == (c_out, s * s * c_in) and got[4:] == (n // s, m // s)
        for k, k2 in ((kh, got[2]), (kw, got[3])):
            Y = [(t - (k - 1) // 2) // s for t in range(k)]
            lo, hi = -((k2 - 1) // 2), k2 // 2
            assert lo <= min(Y) and max(Y) <= hi
            assert k2 == 1 or lo == min(Y) or hi == max(Y)   # no larger than needed
        if s == 1:
            assert got == spec
    assert call((64, 64, 3, 3, 32, 32), 2)[1][2:4] == (3, 3)
    assert call((64, 3, 7, 7, 224, 224), 2)[1][2:4] == (5, 5)
    for spec, s in [((4, 4, 3, 3, 9, 8), 2), ((4, 4, 3, 3, 8, 8), 0), ((4, 4, 9, 3, 8, 8), 2),
                    ((0, 4, 3, 3, 8, 8), 2)]:
        assert call(spec, s)[0] == _lib.LFA_ERR_INVALID_ARG
    assert lib.lfa_crystal_weights(ctypes.byref(_lib.LfaLayer(4, 4, 3, 3, 8, 8)), 2, 0, None, None, 0, None) \
        == _lib.LFA_ERR_INVALID_ARG
    assert lib.lfa_crystal_weights(ctypes.byref(_lib.LfaLayer(4, 4, 3, 3, 8, 8)), 2, 0, ctypes.c_void_p(8),
                                   ctypes.c_void_p(8), 7, None) == _lib.LFA_ERR_INVALID_ARG


@needs_lib
def test_apply_and_lift_reject_bad_arguments_before_touching_the_gpu():
    """lfa_apply, lfa_apply_workspace_bytes and lfa_lift validate on the host:
    layer, kind, level, counts and pointers; empty calls succeed without a
    device."""
    plan = lfa.Plan([lfa.LayerSpec(8, 4, 3, 3, 6, 4)], want_u=True, want_v=True)
    lib, h = plan.lib, plan.handle
    nb = ctypes.c_size_t()
    assert lib.lfa_apply_workspace_bytes(h, 0, 3, ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 3 * 6 * 4 * 8 * 2 * 4                  # two complex buffers, max(c) = 8
    assert lib.lfa_apply_workspace_bytes(h, 1, 3, ctypes.byref(nb)) == _lib.LFA_ERR_INVALID_ARG
    assert lib.lfa_apply_workspace_bytes(h, 0, -1, ctypes.byref(nb)) == _lib.LFA_ERR_INVALID_ARG
    p = ctypes.c_void_p(8)

    def apply(layer=0, kind=0, param=0.0, batch=1, ptr=p, ws_bytes=1 << 30):
        return lib.lfa_apply(h, layer, ptr, ptr, ptr, kind, param, ptr, ptr, batch, ptr,
                             ctypes.c_size_t(ws_bytes), None)

    assert apply(layer=2) == _lib.LFA_ERR_INVALID_ARG
    assert apply(kind=4) == _lib.LFA_ERR_INVALID_ARG
    assert apply(kind=-1) == _lib.LFA_ERR_INVALID_ARG
    assert apply(param=-1.0) == _lib.LFA_ERR_INVALID_ARG
    assert apply(param=float("nan")) == _lib.LFA_ERR_INVALID_ARG
    assert apply(batch=-2) == _lib.LFA_ERR_INVALID_ARG
    assert apply(batch=0) == 0
    assert apply(ptr=ctypes.c_void_p(None)) == _lib.LFA_ERR_INVALID_ARG
    assert apply(ws_bytes=16) == _lib.LFA_ERR_WORKSPACE
    assert _lib.LFA_SPECTRAL_TRUNCATE == 3

    def lift(layer=0, U=p, V=p, idx=p, count=1, uh=p, vh=p):
        return lib.lfa_lift(h, layer, U, V, idx, count, uh, vh, None)

    assert lift(layer=1) == _lib.LFA_ERR_INVALID_ARG
    assert lift(count=-1) == _lib.LFA_ERR_INVALID_ARG
    assert lift(U=None) == _lib.LFA_ERR_INVALID_ARG                 # u_hat without U
    assert lift(V=None) == _lib.LFA_ERR_INVALID_ARG
    assert lift(idx=None) == _lib.LFA_ERR_INVALID_ARG
    assert lift(count=0) == 0
    assert lift(uh=None, vh=None) == 0                              # nothing to write


def test_work_queue_loop_runs_the_hand_over_on_every_trip():
    """Static check of the built work-queue kernels (tests/queue_loop.py):
    in every wave_queue_kernel instance, each loop around the read of the
    next group's code also contains thread 0's queue pop.  A loop structure
    in which the other threads loop around the group code without passing
    the hand-over (a thread-0 region at the bottom of the loop with a
    per-lane exit test) hung the GPU; the check flags all 24 instances of
    that structure and passes the current kernels."""
    import queue_loop

    obj = os.path.join(ROOT, "_build", "jacobi_wave.hip.o")
    if not queue_loop.tools_available() or not os.path.exists(obj):
        pytest.skip("needs the ROCm LLVM tools and the built _build/jacobi_wave.hip.o")
    res = queue_loop.check_object(obj)
    assert len(res) == 24, sorted(res)
    bad = {k: msg for k, (ok, msg) in res.items() if not ok}
    assert not bad, bad


def test_binding_constants_match_header():
    """Every numeric enum constant of include/lfa.h that the binding also
    defines (status codes, flags, info words) has the same value there."""
    import re
    text = open(HEADER).read()
    consts = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(LFA_[A-Z0-9_]+)\s*=\s*(-?\d+)u?\b", text)}
    checked = 0
    for name, val in consts.items():
        if hasattr(_lib, name):
            assert getattr(_lib, name) == val, (name, getattr(_lib, name), val)
            checked += 1
    assert checked >= 20 and _lib.LFA_INFO_WORDS == _lib.LFA_INFO_HIST + _lib.LFA_INFO_HIST_BINS


@needs_lib
def test_info_status_and_sweep_cap_validation():
    """lfa_info_status turns a host copy of the info record into warning
    bits; lfa_plan_set_max_sweeps accepts 1 .. 40 only (no GPU needed)."""
    lib = _lib.load()
    w = _lib.LFA_INFO_WORDS
    info = (ctypes.c_int32 * (2 * w))()
    info[1], info[2], info[w + 1], info[w + 2] = 3, 10, 5, 40
    info[_lib.LFA_INFO_HIST + 3] = 2                 # histogram words carry no warning
    assert lib.lfa_info_status(info, 1) == 0
    assert lib.lfa_info_status(info, 2) == 0
    info[w] = 2                                      # layer 1: two symbols hit the cap
    assert lib.lfa_info_status(info, 2) == _lib.LFA_WARN_NOT_CONVERGED
    info[w + 3] = 1 | 2                              # non-finite and a team time-out
    assert lib.lfa_info_status(info, 2) == (_lib.LFA_WARN_NOT_CONVERGED | _lib.LFA_WARN_NONFINITE
                                            | _lib.LFA_WARN_TEAM_TIMEOUT)
    assert lib.lfa_info_status(None, 1) == _lib.LFA_ERR_INVALID_ARG
    assert lib.lfa_info_status(info, 0) == _lib.LFA_ERR_INVALID_ARG
    plan = lfa.Plan([lfa.LayerSpec(8, 8, 3, 3, 6, 6)])
    for bad in (0, -1, 41):
        assert lib.lfa_plan_set_max_sweeps(plan.handle, bad) == _lib.LFA_ERR_INVALID_ARG
    for good in (1, 7, 40):
        assert lib.lfa_plan_set_max_sweeps(plan.handle, good) == _lib.LFA_OK
    assert lib.lfa_plan_prepare(plan.handle, -1) == _lib.LFA_ERR_INVALID_ARG
