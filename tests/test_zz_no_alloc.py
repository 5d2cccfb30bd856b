"""lfa_svd_noalloc (the entry point that allocates nothing: its scratch is a
static device array of the library) against lfa_svd, through the C ABI."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import banner, to_np

pytestmark = pytest.mark.gpu

DEV = "cuda"


def lfa():
    import paper_2506_05617_amd as m
    return m


def _run_both(L, W, dtype, vectors):
    spec = lfa().LayerSpec(L.c_out, L.c_in, L.kh, L.kw, L.n, L.m)
    plan = lfa().Plan([spec], dtype, want_u=vectors, want_v=vectors)
    Wt = torch.from_numpy(np.ascontiguousarray(W)).to(DEV)
    S1, U1, V1, i1 = plan.svd([Wt])
    S2, U2, V2, i2 = plan.svd_noalloc([Wt])
    torch.cuda.synchronize()
    return plan, (S1[0], U1[0], V1[0], i1), (S2[0], U2[0], V2[0], i2)


def test_noalloc_matches_lfa_svd_twice_then_a_smaller_input():
    """Two calls in a row: the 64 -> 64 channel 64x64-grid layer with U and V
    (whose lfa_svd launch uses the work queue, which does not fit the static
    scratch: the no-allocation call runs the plain launch, bitwise the same),
    then a smaller 16 -> 16 channel 8x8-grid layer in FP64 with vectors.
    Each against lfa_svd elementwise (bitwise) and against the oracle."""
    for case, (L, W), dtype in (
            ("64x64 n=64 uv", workloads.single_layer_64(), torch.float32),
            ("16x16 n=8 fp64 uv", workloads.random_layer(16, 16, 3, 3, 8, 8, seed=91, dtype=np.float64),
             torch.float64)):
        banner(f"noalloc {case}")
        plan, ref, got = _run_both(L, W, dtype, True)
        for a, b, name in zip(ref[:3], got[:3], ("sigma", "U", "V")):
            assert torch.equal(a, b), f"{case}: {name} differs from lfa_svd"
        assert torch.equal(ref[3], got[3]), f"{case}: info differs"
        assert plan.info_status(got[3]) == 0
        fr = np.array([[0, 0], [1, 3], [L.n - 1, L.m // 2], [L.n // 2, 1]])
        S_ref = oracle.lfa_svd(W.astype(np.float64), L.n, L.m, freqs=fr)
        gate = 1e-5 if dtype == torch.float32 else 1e-12
        assert oracle.sigma_error(to_np(got[0])[fr[:, 0], fr[:, 1]], S_ref) <= gate


def test_noalloc_rejects_a_plan_beyond_the_scratch():
    """The 512 x 256 layer keeps every symbol in a global slot (1 GiB): more
    than the 64 MiB scratch, refused with LFA_ERR_WORKSPACE before any launch."""
    banner("noalloc too large")
    spec = lfa().LayerSpec(512, 256, 3, 3, 32, 32)
    plan = lfa().Plan([spec])
    Wt = torch.zeros(512, 256, 3, 3, device=DEV)
    with pytest.raises(lfa().LfaError) as err:
        plan.svd_noalloc([Wt])
    assert err.value.status == lfa()._lib.LFA_ERR_WORKSPACE
