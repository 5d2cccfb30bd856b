"""Failure reporting and capture behaviour of the C ABI on the GPU: non-finite
weights, the plan's sweep cap, and compute calls captured into a graph after
lfa_plan_prepare.  Expected values come from the oracle."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import banner, grad_errors, to_np

pytestmark = pytest.mark.gpu

DEV = "cuda"


def lfa():
    import paper_2506_05617_amd as m
    return m


def _w(W):
    return torch.from_numpy(np.ascontiguousarray(W)).to(DEV)


def _spec(l):
    return lfa().LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m)


# (c_out, c_in, n): the register kernel (<= 64 rows) and the blocked kernel
STATUS_CASES = [(64, 64, 8), (160, 96, 4)]


@pytest.mark.parametrize("case", STATUS_CASES)
def test_nonfinite_weights_are_reported(case):
    """A NaN weight poisons one entry of every symbol of its layer: the call
    ends normally, the layer's info word has the non-finite bit and
    lfa_info_status reports LFA_WARN_NONFINITE; a finite layer of the same
    plan is unaffected (sigma within the gate, no warning bits)."""
    c_out, c_in, n = case
    banner(f"nonfinite {case}")
    Lb, Wb = workloads.random_layer(c_out, c_in, 3, 3, n, n, seed=71)
    Lg, Wg = workloads.random_layer(c_out, c_in, 3, 3, n, n, seed=72)
    Wb = Wb.copy()
    Wb[1, 2, 1, 1] = np.nan
    plan = lfa().Plan([_spec(Lb), _spec(Lg)])
    S, _, _, info = plan.svd([_w(Wb), _w(Wg)])
    torch.cuda.synchronize()
    inf = to_np(info)
    assert inf[0, 3] & 1, inf
    assert inf[1, 3] == 0 and inf[1, 0] == 0, inf
    st = plan.info_status(info)
    assert st & lfa()._lib.LFA_WARN_NONFINITE, st
    assert not np.all(np.isfinite(to_np(S[0])))
    S_ref = oracle.lfa_svd(Wg.astype(np.float64), n, n)
    assert oracle.sigma_error(to_np(S[1]), S_ref) <= 1e-5
    assert plan.info_status(info[1:]) == 0


@pytest.mark.parametrize("case", STATUS_CASES + [(64, 64, 64)])
def test_sweep_cap_reports_nonconverged(case):
    """With the plan's sweep cap at 2 no symbol converges: every decomposed
    symbol is counted in LFA_INFO_NONCONVERGED, no symbol ran more than 2
    sweeps, lfa_info_status reports LFA_WARN_NOT_CONVERGED and the outputs
    are finite.  (64, 64, 64) runs the register kernel's work queue.)  Back
    at the default cap the same plan converges within the gate."""
    c_out, c_in, n = case
    banner(f"sweep cap {case}")
    L, W = workloads.random_layer(c_out, c_in, 3, 3, n, n, seed=73)
    plan = lfa().Plan([_spec(L)])
    Wt = _w(W)
    plan.set_max_sweeps(2)
    S, _, _, info = plan.svd([Wt])
    torch.cuda.synchronize()
    inf = to_np(info)[0]
    canon = n // 2 + 1 + (n // 2 - 1) * n + (n // 2 + 1)      # one symbol per conjugate pair
    assert inf[0] == canon and inf[1] == 2, inf
    hist = inf[lfa()._lib.LFA_INFO_HIST:]
    assert hist[2] == canon and hist.sum() == canon, hist      # every symbol in the bin of the cap
    assert plan.info_status(info) & lfa()._lib.LFA_WARN_NOT_CONVERGED
    assert np.all(np.isfinite(to_np(S[0])))
    plan.set_max_sweeps(40)
    S, _, _, info = plan.svd([Wt])
    torch.cuda.synchronize()
    assert to_np(info)[0, 0] == 0 and plan.info_status(info) == 0
    fr = np.array([[0, 0], [1, 2], [n - 1, n // 2]])
    S_ref = oracle.lfa_svd(W.astype(np.float64), n, n, freqs=fr)
    assert oracle.sigma_error(to_np(S[0])[fr[:, 0], fr[:, 1]], S_ref) <= 1e-5
    with pytest.raises(lfa().LfaError):
        plan.set_max_sweeps(41)


def test_prepared_plan_captures_into_a_torch_graph():
    """After lfa_plan_prepare(plan, k) the persistent sigma-only SVD, top-k
    and persistent sigma gradient capture into a torch CUDA graph (no upload
    or allocation inside the capture); three replays with new weights and
    eager work in between each match the oracle.  A k the plan was not
    prepared for is refused under capture with LFA_ERR_NOT_PREPARED."""
    banner("capture after prepare")
    shapes = ((3, 16, 8), (16, 32, 4), (32, 96, 3))
    layers, Ws = workloads.resnet18_stack(seed=81, shapes=shapes)
    plan = lfa().Plan([_spec(l) for l in layers])
    k = 4
    plan.prepare(k)
    Wt = [_w(W) for W in Ws]
    S, _, _ = plan._alloc_outputs(Wt[0].device, False, False)
    info = torch.zeros(len(layers), lfa()._lib.LFA_INFO_WORDS, dtype=torch.int32, device=DEV)
    g = torch.ones(len(layers), k, device=DEV)
    dW = [torch.empty_like(W) for W in Wt]
    plan.workspace(Wt[0].device)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            plan.svd(Wt, persistent=True, info=info, out=(S, [None] * 3, [None] * 3))
            vals, idx = plan.topk(S, k)
            plan.sigma_grad(Wt, idx, g, out=dW, persistent=True)
    torch.cuda.current_stream().wait_stream(side)
    rng = np.random.default_rng(8)
    for rep in range(3):
        news = [(rng.standard_normal(W.shape) * 0.2).astype(np.float32) for W in Ws]
        for W, x in zip(Wt, news):
            W.copy_(torch.from_numpy(x))
        graph.replay()
        torch.cuda.synchronize()
        assert plan.info_status(info) == 0
        v, ix = to_np(vals), to_np(idx)
        for li, l in enumerate(layers):
            W64 = news[li].astype(np.float64)
            s_ref = oracle.lfa_svd(W64, l.n, l.m)
            ov, _ = oracle.topk(s_ref, k)
            np.testing.assert_allclose(v[li], ov, rtol=0, atol=1e-5 * ov[0])
            S_sym = oracle.lfa_svd(W64, l.n, l.m, freqs=ix[li][:, :2])
            ref = oracle.sigma_grad(W64, l.n, l.m, ix[li], np.ones(k))
            grad_errors(to_np(dW[li]), ref, S_sym, ix[li], None, f"captured replay {rep} layer {li}")
        plan.topk(S, k)            # eager work between the replays
        torch.cuda.synchronize()
    # a new k needs an upload: refused while capturing
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(lfa().LfaError) as err:
        with torch.cuda.stream(side):
            with torch.cuda.graph(g2, stream=side):
                dW[0].zero_()
                plan.sigma_grad(Wt, idx[:, :2].contiguous(), g[:, :2].contiguous(), out=dW, persistent=True)
    assert err.value.status == lfa()._lib.LFA_ERR_NOT_PREPARED
    torch.cuda.synchronize()


def test_persistent_busy_records_match_the_launch():
    """lfa_svd_persistent_busy: the same singular values as
    lfa_svd_persistent (bitwise), one record per work-group of the launch,
    items taken summing to the work list, busy time within the launch, and
    compute-unit identities that are few per work-group (at most a few
    work-groups share a compute unit)."""
    banner("persistent busy records")
    layers, Ws = workloads.resnet18_stack(seed=85, shapes=((3, 64, 8), (64, 64, 8), (64, 128, 4), (128, 256, 3)))
    plan = lfa().Plan([_spec(l) for l in layers])
    Wt = [_w(W) for W in Ws]
    S1, _, _, _ = plan.svd(Wt, persistent=True)
    S2, _, _, info, rec = plan.persistent_busy(Wt)
    torch.cuda.synchronize()
    for a, b in zip(S1, S2):
        assert torch.equal(a, b)
    rec = to_np(rec)
    assert rec.shape[1] == 4 and rec.shape[0] >= 1
    assert np.all(rec[:, 0] >= 0) and np.all(rec[:, 1] >= 0)
    assert rec[:, 1].sum() > 0
    cus = {(int(x), int(h)) for x, h in rec[:, 2:]}
    assert len(cus) >= 1 and rec.shape[0] <= 8 * len(cus)


HIST_CASES = [
    # c_out, c_in, n, persistent: register kernel (work queue), register /
    # blocked kernels, and the persistent launch
    (64, 64, 64, False),
    (160, 96, 8, False),
    (24, 40, 12, False),
    (160, 96, 8, True),
]


@pytest.mark.parametrize("case", HIST_CASES)
def test_sweep_histogram_is_consistent(case):
    """The info record's sweep histogram counts every decomposed symbol once
    (one per conjugate pair), its weighted sum is the sweep total and its
    last nonzero bin the sweep maximum."""
    c_out, c_in, n, persistent = case
    banner(f"sweep histogram {case}")
    L, W = workloads.random_layer(c_out, c_in, 3, 3, n, n, seed=74)
    plan = lfa().Plan([_spec(L)])
    S, _, _, info = plan.svd([_w(W)], persistent=persistent)
    torch.cuda.synchronize()
    inf = to_np(info)[0]
    lib = lfa()._lib
    hist = inf[lib.LFA_INFO_HIST:lib.LFA_INFO_HIST + lib.LFA_INFO_HIST_BINS]
    canon = (n * n + 4) // 2 if n % 2 == 0 else (n * n + 1) // 2
    assert hist.sum() == canon, (hist, canon)
    assert int(np.dot(np.arange(len(hist)), hist)) == inf[lib.LFA_INFO_SUM_SWEEPS], (hist, inf)
    assert np.flatnonzero(hist).max() == inf[lib.LFA_INFO_MAX_SWEEPS], (hist, inf)
    assert inf[lib.LFA_INFO_NONCONVERGED] == 0



def test_phase_record():
    """The register kernel's phase record: with a buffer set, a launch adds
    positive work-group time to the load, sweep and finish phases (and to
    the saves of the work queue when it runs), with the sweeps the largest;
    after record_phases(None) a launch adds nothing; σ is unchanged."""
    banner("phase record")
    L, W = workloads.random_layer(64, 64, 3, 3, 64, 64, seed=75)
    plan = lfa().Plan([_spec(L)], want_u=True, want_v=True)
    Wt = _w(W)
    S0 = plan.svd([Wt])[0][0].clone()
    ticks = torch.zeros(4, dtype=torch.int64, device=DEV)
    plan.record_phases(ticks)
    S1 = plan.svd([Wt])[0][0]
    torch.cuda.synchronize()
    plan.record_phases(None)
    tk = ticks.cpu().numpy()
    assert np.all(tk[:3] > 0), tk
    assert tk[1] > tk[0] and tk[1] > tk[2], tk
    if plan.queue_info(0)[0] > 0:
        assert tk[3] > 0, tk
    assert torch.equal(S0, S1)
    before = ticks.clone()
    plan.svd([Wt])
    torch.cuda.synchronize()
    assert torch.equal(ticks, before)
