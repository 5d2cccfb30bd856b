"""Benchmark of the LFA SVD hot path on one MI355X.

Headline (``value``): singular values per second, with left and right
singular vectors, for the 64 -> 64 channel, 3x3, 64x64-grid layer
(4096 symbols of 64x64): one step = symbol assembly + Jacobi SVD + sort /
normalise / write of sigma, U, V (one lfa_svd call; weights resident in HBM,
outputs preallocated).

Also reported (``workloads``):
  * 16 -> 16 channels on a 32x32 grid in FP64 mode (sigma, U, V);
  * 256 -> 512 channels on a 32x32 grid (1024 symbols of 512x256), sigma-only
    and with U, V, plus the instance with rank-one taps;
  * the 12-layer ResNet-18-shaped stack: sigma-gradient throughput in layers/s
    (forward sigma of every layer, top-8 per layer, dL/dW), batched (a HIP
    graph of one persistent SVD launch keeping U and V, top-8 and one adjoint
    launch) and plain (one launch per layer and stage);
  * 64 -> 64 channels, 7x7 kernel, 224x224 grid (50176 symbols), sigma-only,
    with FP32 fused assembly and with split-BF16 matrix-core assembly
    (3 and 6 products), and the assembly kernel alone against HBM bandwidth.
The roofline of the headline's dominant kernel (the fused SVD kernel) is
algorithmic FLOP per launch (sweeps measured by the kernel x pairs x
per-pair work) over the launch time measured with HIP events.  The FP64
oracle (NumPy/LAPACK) is timed on the host cores on the headline layer; the
same leg reports every workload's sigma error against the oracle.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--quick]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2506_05617_amd as lfa  # noqa: E402
import workloads  # noqa: E402

METRIC = "singular values/s (with vectors) and σ-grad layers/s vs plain at σ rel err ≤1e-5"
PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X, packed FP32 (the kernels are compiled without packed FP32: half that)
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the headline kernel from the PMC passes recorded in
# profiles/wave_queue_kernel_single_layer_64x64_uv.md (FETCH_SIZE x 2.00 +
# WRITE_SIZE x 1.00, calibrated with a copy of known size), valid only for the
# kernel source they were taken on.
HEAD_TRAFFIC = {"bytes": 154.12e6 + 430.67e6, "source_hash": "dbb3f0c77c1e297e",
                "files": ("jacobi_device.hpp", "jacobi_wave.hip", "lfa_internal.hpp", "api.cpp")}


# The paper's LFA wall-clock times for c = 16 (sigma only; Xeon Gold 6242,
# 16 cores, NumPy), Table II: context for the paper-scale workload.
PAPER_TABLE2_SECONDS = {256: 2.30, 512: 8.49, 1024: 33.01, 2048: 130.20, 4096: 520.21,
                        8192: 2077.44, 16384: 7521.93}


def source_hash(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2506_05617_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def jacobi_flops(layer, sum_sweeps: int, vectors: bool) -> float:
    """Algorithmic FLOP of the one-sided Jacobi sweeps: per column pair and
    sweep, three inner products over the M rows (16 M) and the complex
    rotation of two columns of G (20 M) and, with vectors, of the
    accumulator (20 N); N(N-1)/2 pairs per sweep.  sum_sweeps counts the
    sweeps of the symbols actually decomposed."""
    M, N = max(layer.c_out, layer.c_in), min(layer.c_out, layer.c_in)
    per_pair = 36.0 * M + (20.0 * N if vectors else 0.0)
    return sum_sweeps * N * (N - 1) / 2.0 * per_pair


def event_times(fn, steps, warmup):
    """Per-call times from HIP events on the current stream, and wall time."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        fn()
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [s.elapsed_time(e) for s, e in zip(starts, ends)]


def run_strided(L, stride, W, dev, steps, warmup):
    """A stride-`stride` layer through its crystal form: weight repack and
    SVD (sigma + U + V) of the coarse stride-1 layer, per step."""
    Wt = torch.from_numpy(W).to(dev)
    spec = lfa.LayerSpec(L.c_out, L.c_in, L.kh, L.kw, L.n, L.m)
    c = lfa.crystal_layer(spec, stride)
    plan = lfa.Plan([c], torch.float32, want_u=True, want_v=True)
    S, U, V = plan._alloc_outputs(dev, True, True)
    info = torch.zeros(1, lfa._lib.LFA_INFO_WORDS, dtype=torch.int32, device=dev)

    def step():
        Wc = lfa.crystal_weights(Wt, spec, stride)
        plan.svd([Wc], info=info, out=(S, U, V))

    wall, ev = event_times(step, steps, warmup)
    inf = info.cpu().numpy()[0]
    ms = wall * 1e3 / steps
    nsig = c.n * c.m * min(c.c_out, c.c_in)
    return dict(layer=L, stride=stride, crystal=c, W=W, S=S[0], ms=ms, kernel_ms=float(np.mean(ev)),
                info=[int(x) for x in inf], sigma_per_s=nsig / (ms * 1e-3))


def run_layer(L, W, dev, vectors, steps, warmup, asm=None, dtype=torch.float32):
    Wt = torch.from_numpy(W).to(dev)
    spec = lfa.LayerSpec(L.c_out, L.c_in, L.kh, L.kw, L.n, L.m)
    plan = lfa.Plan([spec], dtype, want_u=vectors, want_v=vectors, asm=asm)
    S, U, V = plan._alloc_outputs(dev, vectors, vectors)
    info = torch.zeros(1, lfa._lib.LFA_INFO_WORDS, dtype=torch.int32, device=dev)

    def step():
        plan.svd([Wt], info=info, out=(S, U, V))

    wall, ev = event_times(step, steps, warmup)
    inf = info.cpu().numpy()[0]
    ms = wall * 1e3 / steps
    qr = plan.preconditioned(0)
    # QR preconditioning: the sweeps run on the N x N factors
    Lj = workloads.Layer(L.r, L.r, 1, 1, L.n, L.m) if qr else L
    return dict(layer=L, W=W, S=S[0], U=U[0], V=V[0], ms=ms, kernel_ms=float(np.mean(ev)),
                info=[int(x) for x in inf], sigma_per_s=L.num_sigma / (ms * 1e-3),
                flops=jacobi_flops(Lj, int(inf[2]), vectors), plan=plan, qr=qr)


def bench_stack(dev, steps):
    """The ResNet-18 stack's sigma-gradient step: forward sigma of every
    symbol of every layer, top-8 per layer, dL/dW of the top-8 sum.

    Batched: one HIP graph of [persistent SVD keeping U of every symbol (the
    side the working matrix converges to: no rotation accumulator) -> top-8
    -> one-sided adjoint (V of each pick recomputed from W)].  Plain: the same
    algorithm eagerly, one SVD launch per layer (lfa_svd), then lfa_topk and
    lfa_adjoint_onesided.  Also timed: the graph keeping U and V of every
    symbol, the sigma-only graph (vectors of the picks recomputed by a second
    SVD), and the eager sigma-only path with per-layer recomputation."""
    layers, Ws = workloads.resnet18_stack()
    specs = [lfa.LayerSpec(l.c_out, l.c_in, l.kh, l.kw, l.n, l.m) for l in layers]
    plan = lfa.Plan(specs, torch.float32)
    plan_u = lfa.Plan(specs, torch.float32, want_u=True)
    Wt = [torch.from_numpy(w).to(dev) for w in Ws]
    k = 8
    ones = torch.ones(len(specs), k, device=dev)
    S, _, _ = plan._alloc_outputs(dev, False, False)
    Su, Uu, _ = plan_u._alloc_outputs(dev, True, False)
    dWu = [torch.empty_like(W) for W in Wt]
    info = torch.zeros(len(specs), lfa._lib.LFA_INFO_WORDS, dtype=torch.int32, device=dev)
    none = [None] * len(S)
    res = {}

    def plain():
        plan_u.svd(Wt, persistent=False, info=info, out=(Su, Uu, none))
        vals, idx = plan_u.topk(Su, k)
        res["plain"] = (vals, idx, plan_u.adjoint_onesided(Wt, Su, Uu, idx, ones, out=dWu))

    def plain_recompute():
        plan.svd(Wt, persistent=False, info=info, out=(S, none, none))
        vals, idx = plan.topk(S, k)
        plan.sigma_grad(Wt, idx, ones)

    graph = lfa.GraphStep(plan_u, Wt, k)
    graph_uv = lfa.GraphStep(lfa.Plan(specs, torch.float32, want_u=True, want_v=True), Wt, k)
    graph_s = lfa.GraphStep(plan, Wt, k)

    def replay(g):
        g.replay()

    wall_p, _ = event_times(plain, steps, 1)
    wall_r, _ = event_times(plain_recompute, steps, 1)
    wall_b, _ = event_times(lambda: replay(graph), steps, 1)
    wall_uv, _ = event_times(lambda: replay(graph_uv), steps, 1)
    wall_s, _ = event_times(lambda: replay(graph_s), steps, 1)
    torch.cuda.synchronize()
    # the same two steps with the autotuner's choices (a fresh JSON cache:
    # every choice is timed here); the graph is captured after tuning
    import tempfile

    t0 = time.perf_counter()
    with tempfile.TemporaryDirectory() as tmp:
        plan_u.autotune(Wt, os.path.join(tmp, "lfa_tune.json"))
    tune_s = time.perf_counter() - t0
    graph_t = lfa.GraphStep(plan_u, Wt, k)
    wall_pt, _ = event_times(plain, steps, 1)
    wall_bt, _ = event_times(lambda: replay(graph_t), steps, 1)
    torch.cuda.synchronize()
    tuned = dict(plain_ms=wall_pt * 1e3 / steps, batched_ms=wall_bt * 1e3 / steps, tune_s=tune_s,
                 layer_choices=[list(plan_u.tuning(i)) for i in range(len(specs))],
                 cost_model=list(plan_u.cost_model()))
    if wall_bt < wall_b:
        graph, wall_b = graph_t, wall_bt
    if wall_pt < wall_p:
        wall_p = wall_pt
    batched_out = (graph.vals.clone(), graph.idx.clone(), [d.clone() for d in graph.dW])
    nl = len(specs)
    # the batched step against the FP32 roofline: algorithmic flops of the
    # one-sided forward sweeps (working matrix only, no accumulator) over the
    # step time; and the load balance of its persistent launch, from one
    # instrumented launch (busy time of every compute unit over the launch)
    info_b = graph.info.cpu().numpy()
    flops = sum(jacobi_flops(l, int(info_b[i][2]), False) for i, l in enumerate(layers))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, _, _, _, rec = plan_u.persistent_busy(Wt)
    e1.record()
    torch.cuda.synchronize()
    span_s = e0.elapsed_time(e1) * 1e-3
    rec = rec.cpu().numpy()
    per_cu = {}
    for busy_t, items, xcc, hw in rec:
        if items == 0 and busy_t == 0:
            continue
        key = (int(xcc), int(hw))
        b, c = per_cu.get(key, (0, 0))
        per_cu[key] = (b + busy_t * 1e-8, c + 1)
    frac = np.array([b / (span_s * c) for b, c in per_cu.values()])
    balance = dict(compute_units=len(per_cu), work_groups=int(sum(c for _, c in per_cu.values())),
                   launch_ms=span_s * 1e3, busy_frac_min=float(frac.min()), busy_frac_median=float(np.median(frac)),
                   busy_frac_mean=float(frac.mean()), busy_frac_max=float(frac.max()))
    roof = dict(algorithmic_gflop=flops / 1e9, tflops=flops / (wall_b / steps) / 1e12,
                frac_of_fp32_peak=flops / (wall_b / steps) / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                sweeps_sum=[int(x) for x in info_b[:, 2]], per_cu_busy=balance)
    return dict(layers=layers, Ws=Ws, graph=graph, plain_out=res["plain"], batched_out=batched_out, S=Su,
                plain_layers_per_s=nl * steps / wall_p, batched_layers_per_s=nl * steps / wall_b,
                plain_ms=wall_p * 1e3 / steps, batched_ms=wall_b * 1e3 / steps,
                plain_sigma_only_recompute_ms=wall_r * 1e3 / steps, tuned=tuned, roofline=roof,
                batched_uv_graph_ms=wall_uv * 1e3 / steps,
                batched_sigma_only_ms=wall_s * 1e3 / steps)


def bench_assembly(dev, steps, asm):
    """The assembly kernel alone on the 224x224, 7x7 layer: 1.64 GB of
    symbols written; HBM-bound."""
    L, W, _ = workloads.large_grid_7x7()
    Wt = torch.from_numpy(W).to(dev)
    plan = lfa.Plan([lfa.LayerSpec(L.c_out, L.c_in, L.kh, L.kw, L.n, L.m)], asm=asm)
    out = {}

    def step():
        out["A"] = plan.symbols([Wt])[0]

    step()
    torch.cuda.synchronize()
    A = out["A"]
    # reuse the output buffer: time the kernel through the C ABI directly
    w_arr, k0 = lfa._lib.ptr_array([Wt.data_ptr()])
    a_arr, k1 = lfa._lib.ptr_array([A.data_ptr()])
    lib = plan.lib

    def launch():
        lfa._lib.check(lib.lfa_symbols(plan.handle, w_arr, a_arr, lfa.lfa._stream_ptr()), "lfa_symbols")

    _, ev = event_times(launch, steps, 2)
    ms = float(np.mean(ev))
    bytes_moved = A.numel() * A.element_size() + W.nbytes
    return dict(ms=ms, gbs=bytes_moved / (ms * 1e-3) / 1e9, bytes=bytes_moved, A=A, L=L, W=W)


def bench_split(dev, steps, L, W, vectors):
    """Assembly and SVD timed apart, as the paper's Table III splits its
    runtime into the transformation and the SVD: lfa_symbols (materialised
    symbols), lfa_svd_symbols on them, and the fused lfa_svd that never
    writes the symbols."""
    Wt = torch.from_numpy(W).to(dev)
    plan = lfa.Plan([lfa.LayerSpec(L.c_out, L.c_in, L.kh, L.kw, L.n, L.m)], want_u=vectors, want_v=vectors)
    A = plan.symbols([Wt])[0]
    torch.cuda.synchronize()
    w_arr, k0 = lfa._lib.ptr_array([Wt.data_ptr()])
    a_arr, k1 = lfa._lib.ptr_array([A.data_ptr()])

    def asm():
        lfa._lib.check(plan.lib.lfa_symbols(plan.handle, w_arr, a_arr, lfa.lfa._stream_ptr()), "lfa_symbols")

    _, ev_asm = event_times(asm, steps, 2)
    _, ev_svd = event_times(lambda: plan.svd_symbols([A]), steps, 2)
    S, U, V = plan._alloc_outputs(dev, vectors, vectors)
    _, ev_fused = event_times(lambda: plan.svd([Wt], out=(S, U, V)), steps, 2)
    t_asm, t_svd, t_fused = (float(np.mean(e)) for e in (ev_asm, ev_svd, ev_fused))
    # the fused kernel's own split: work-group time in each phase (the
    # register kernel's phase record), apportioning the fused launch
    ticks = torch.zeros(4, dtype=torch.int64, device=dev)
    plan.record_phases(ticks)
    plan.svd([Wt], out=(S, U, V))
    torch.cuda.synchronize()
    plan.record_phases(None)
    tk = ticks.cpu().numpy().astype(np.float64)
    share = tk / max(tk.sum(), 1.0)
    phases = dict(zip(("load_asm", "sweeps", "post", "queue_save"), share.tolist()))
    return dict(asm_ms=t_asm, svd_ms=t_svd, asm_share=t_asm / (t_asm + t_svd), fused_ms=t_fused,
                vectors=vectors, fused_phase_share=phases,
                fused_phase_ms={k: v * t_fused for k, v in phases.items()})


def bench_apply(head, dev, kind, batch=8, steps=10):
    """A spectral function of the headline layer's operator applied to
    `batch` images through its SVD (lfa_apply: forward transforms, the
    per-frequency map U f(S) V^* or V f(S) U^*, inverse transforms).  The
    per-frequency map reads U and V once for the batch: HBM-bound."""
    L, plan = head["layer"], head["plan"]
    S, U, V = head["S"], head["U"], head["V"]
    rng = np.random.default_rng(7)
    cx = L.c_out if kind == "pinv" else L.c_in
    x = torch.from_numpy(rng.standard_normal((batch, cx, L.n, L.m)).astype(np.float32)).to(dev)
    param = 0.0
    out = {}

    def step():
        out["y"] = plan.apply(0, S, U, V, x, kind, param)

    _, ev = event_times(step, steps, 2)
    ms = float(np.mean(ev))
    y = out["y"]
    bytes_moved = (U.numel() * U.element_size() + V.numel() * V.element_size() + S.numel() * S.element_size()
                   + x.numel() * x.element_size() + y.numel() * y.element_size())
    return dict(ms=ms, gbs=bytes_moved / (ms * 1e-3) / 1e9, bytes=bytes_moved, x=x, y=y, kind=kind,
                param=param, W=head["W"], layer=L, batch=batch)


def cpu_leg(head, extra):
    """FP64 oracle on the host: timed on the headline layer (all 4096 symbols,
    sigma+U+V, thread pool over frequency chunks, one BLAS thread each), and
    used to report the sigma error of every GPU result."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    import oracle

    L, W = head["layer"], head["W"]
    cores = min(os.cpu_count() or 1, 16)
    pp, qq = np.meshgrid(np.arange(L.n), np.arange(L.m), indexing="ij")
    freqs = np.stack([pp.ravel(), qq.ravel()], axis=1)
    chunks = np.array_split(freqs, cores * 4)
    W64 = W.astype(np.float64)

    def work(fr):
        return fr, oracle.lfa_svd(W64, L.n, L.m, compute_uv=True, freqs=fr)

    # Whole passes over the layer until at least 10 s of wall time (>= 3).
    reps = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while reps < 3 or time.perf_counter() - t0 < 10.0:
            with ThreadPoolExecutor(max_workers=cores) as ex:
                parts = list(ex.map(work, chunks))
            reps += 1
        secs = (time.perf_counter() - t0) / reps
    note(f"oracle timing: {reps} passes, {secs:.3f} s each")
    S_ref = np.zeros((L.n, L.m, L.r))
    for fr, (s, _, _) in parts:
        S_ref[fr[:, 0], fr[:, 1]] = s
    errors = {"single_layer_64": oracle.sigma_error(head["S"].cpu().numpy(), S_ref)}

    rng = np.random.default_rng(0)
    full_cache = {}

    def oracle_full(Wx, n, m):
        """The oracle's singular values of every symbol of a layer (frequency
        chunks over the host threads), cached per weight tensor."""
        key = (id(Wx), n, m)
        if key not in full_cache:
            W64x = Wx.astype(np.float64)
            pq = np.stack([g.ravel() for g in np.meshgrid(np.arange(n), np.arange(m), indexing="ij")], axis=1)
            with threadpool_limits(limits=1), ThreadPoolExecutor(max_workers=cores) as ex:
                parts = list(ex.map(lambda c: oracle.lfa_svd(W64x, n, m, freqs=c),
                                    np.array_split(pq, cores * 8)))
            full_cache[key] = np.concatenate(parts).reshape(n, m, -1)
        return full_cache[key]

    def whole_grid(name, res):
        """sigma error over every symbol of the layer."""
        Lx = res["layer"]
        ref = oracle_full(res["W"], Lx.n, Lx.m)
        got = res["S"].cpu().numpy()
        errors[name] = oracle.sigma_error(got, ref)
        return got, ref

    def sampled(name, res, nsamp=64):
        Lx, Wx = res["layer"], res["W"]
        fr = np.stack([rng.integers(0, Lx.n, nsamp), rng.integers(0, Lx.m, nsamp)], axis=1)
        ref = oracle.lfa_svd(Wx.astype(np.float64), Lx.n, Lx.m, freqs=fr)
        got = res["S"].cpu().numpy()[fr[:, 0], fr[:, 1]]
        errors[name] = oracle.sigma_error(got, ref)
        return got, ref

    with threadpool_limits(limits=cores):
        for name, res in extra.items():
            if name == "stack":
                st = res
                vals, idx, dW = st["plain_out"]
                idx_np = idx.cpu().numpy()
                sig_err = 0.0
                for li, l in enumerate(st["layers"]):
                    sref = oracle_full(st["Ws"][li], l.n, l.m)
                    sig_err = max(sig_err, oracle.sigma_error(st["S"][li].cpu().numpy(), sref))
                    ov, _ = oracle.topk(sref, 8)
                    errors[f"stack_top8_layer{li}"] = float(np.max(np.abs(vals[li].cpu().numpy() - ov)) / ov[0])
                errors["stack_sigma_all_layers"] = sig_err
                # gradient of the top-8 sum against the oracle's for the same
                # picks: elementwise (max |dW - ref| / max |ref|) and
                # Frobenius-relative, worst layer, with the smallest relative
                # gap of a pick to the rest of its symbol
                for tag, (_, ix, d) in (("plain", st["plain_out"]), ("batched", st["batched_out"])):
                    ix = ix.cpu().numpy()
                    e_max = e_fro = 0.0
                    gap = np.inf
                    for li, l in enumerate(st["layers"]):
                        W64l = st["Ws"][li].astype(np.float64)
                        ref = oracle.sigma_grad(W64l, l.n, l.m, ix[li])
                        got = d[li].cpu().numpy().astype(np.float64)
                        e_max = max(e_max, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
                        e_fro = max(e_fro, float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
                        ssym = oracle.lfa_svd(W64l, l.n, l.m, freqs=ix[li][:, :2])
                        for s_, (p_, q_, j_) in enumerate(ix[li]):
                            others = np.delete(ssym[s_], j_)
                            if others.size:
                                gap = min(gap, float(np.min(np.abs(others - ssym[s_][j_])) / ssym[s_][0]))
                    errors[f"stack_{tag}_grad_rel_max"] = e_max
                    errors[f"stack_{tag}_grad_rel_frobenius"] = e_fro
                errors["stack_pick_min_rel_gap"] = gap
            elif name.startswith("rank_one"):
                got, ref = whole_grid(name, res)
                errors[name + "_zero_sigma_max_rel"] = float(np.max(got[..., 9:] / got[..., :1]))
                W64 = res["W"].astype(np.float64)
                Sall = res["S"].cpu().numpy().astype(np.float64)
                Lx = res["layer"]
                errors[name + "_parseval_rel"] = float(abs(np.sum(Sall ** 2) / (Lx.n * Lx.m * np.sum(W64 ** 2)) - 1))
            elif name.startswith("apply"):
                Lx = res["layer"]
                ref = oracle.apply_spectral(res["W"].astype(np.float64), res["x"].cpu().numpy().astype(np.float64),
                                            Lx.n, Lx.m, res["kind"], res["param"])
                errors[name + "_rel_max"] = float(np.max(np.abs(res["y"].cpu().numpy() - ref)) / np.max(np.abs(ref)))
            elif name.startswith("strided"):
                Lx, s = res["layer"], res["stride"]
                A = oracle.crystal_symbols(res["W"].astype(np.float64), Lx.n, Lx.m, s)
                ref = np.linalg.svd(A, compute_uv=False)
                errors[name] = oracle.sigma_error(res["S"].cpu().numpy(), ref)
            elif name.startswith("assembly"):
                fr = np.stack([rng.integers(0, res["L"].n, 32), rng.integers(0, res["L"].m, 32)], axis=1)
                ref = oracle.symbols(res["W"].astype(np.float64), res["L"].n, res["L"].m, fr)
                got = res["A"].cpu().numpy()[fr[:, 0], fr[:, 1]]
                scale = np.max(np.sum(np.abs(res["W"].astype(np.float64)), axis=(2, 3)))
                errors[name + "_symbol_rel"] = float(np.max(np.abs(got - ref)) / scale)
            elif name == "paper_scale_c16_n16384":
                sampled(name, res)          # 1.3e8 symbols: 64 sampled ones
            else:
                whole_grid(name, res)
            note(f"oracle check of {name} done")
    nsig = L.n * L.m * L.r
    return dict(value=nsig / secs, unit="singular values/s", cores=cores, kind="oracle",
                sample=f"all {L.n * L.m} symbols of the 64x64 layer, sigma+U+V, complex128 "
                       f"NumPy/LAPACK, {cores} threads, mean of {reps} passes ({secs:.3f} s each)"), errors


def note(msg):
    """Progress line on stderr; stdout carries only the JSON result."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--only", default=None,
                    help="run only these extra workloads after the headline (comma-separated): apply, fp64, "
                         "rect, strided, split, stack, large, assembly, paper")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the LFA SVD shards over frequencies, but this benchmark "
              "runs and reports a single MI355X only (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lfa.load()

    L, W = workloads.single_layer_64()
    head = run_layer(L, W, dev, True, args.steps, args.warmup)
    note(f"headline: {head['ms']:.3f} ms per step")
    achieved = head["flops"] / (head["kernel_ms"] * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": head["sigma_per_s"],
        "unit": "singular values/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian weights)",
        "config": {"workload": "single conv layer 64->64, 3x3, 64x64 periodic grid, "
                               "4096 symbols 64x64, sigma+U+V",
                   "c_in": 64, "c_out": 64, "kernel": 3, "n": 64, "symbols": 4096},
        "sweeps": {"sum": head["info"][2], "max": head["info"][1], "nonconverged": head["info"][0],
                   "histogram": {str(k): c for k, c in enumerate(
                       head["info"][lfa._lib.LFA_INFO_HIST:lfa._lib.LFA_INFO_HIST + lfa._lib.LFA_INFO_HIST_BINS])
                                 if c}},
        "roofline": {"bound": "alu", "kernel": "wave_queue_kernel_f32<64,64> (work queue of groups, 6 sweeps per turn; fused assembly + Jacobi + sort/write)",
                     "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": (HEAD_TRAFFIC["bytes"]
                                 if source_hash(HEAD_TRAFFIC["files"]) == HEAD_TRAFFIC["source_hash"]
                                 else None),
                     "kernel_ms": head["kernel_ms"]},
    }
    extra = {}
    only = None if args.only is None else set(args.only.split(","))
    sel = (lambda name: only is None or name in only) if not args.quick else (lambda name: False)
    if not args.quick:
        reps = 3
        wl = {}
    if sel("apply"):
        # spectral functions of the headline layer through its SVD (8 images)
        for kind in ("identity", "pinv"):
            a = bench_apply(head, dev, kind)
            extra["apply_" + kind] = a
            wl["apply_64x64_" + kind + "_b8"] = dict(ms=a["ms"], hbm_gbs=a["gbs"],
                                                    frac_of_hbm_peak=a["gbs"] / PEAK_HBM_GBS, batch=a["batch"])
        note("spectral apply done")
    if sel("fp64"):
        L1, W1 = workloads.single_layer_16()
        r = run_layer(L1, W1, dev, True, reps * 3, 1, dtype=torch.float64)
        extra["single_layer_16_fp64"] = r
        wl["single_layer_16_fp64"] = dict(ms=r["ms"], sigma_per_s=r["sigma_per_s"], sweeps=r["info"][1:3],
                                          vectors=True, dtype="f64")
        # the headline layer in FP64 mode (the same float32 weights, upcast)
        r = run_layer(L, W.astype(np.float64), dev, True, reps, 1, dtype=torch.float64)
        extra["single_layer_64_fp64"] = r
        wl["single_layer_64_fp64"] = dict(ms=r["ms"], sigma_per_s=r["sigma_per_s"], sweeps=r["info"][1:3],
                                          vectors=True, dtype="f64")
        note("fp64 single layers done")
    if sel("rect"):
        L3, W3 = workloads.rectangular_256_512()
        for vec in (False, True):
            r = run_layer(L3, W3, dev, vec, reps, 1)
            key = "rectangular_512x256" + ("_uv" if vec else "")
            extra[key] = r
            wl[key] = dict(ms=r["ms"], sigma_per_s=r["sigma_per_s"], sweeps=r["info"][1:3], vectors=vec,
                           qr_preconditioned=r["qr"],
                           tflops=r["flops"] / (r["kernel_ms"] * 1e-3) / 1e12)
        L3r, W3r = workloads.rank_one_taps()
        r = run_layer(L3r, W3r, dev, True, reps, 1)
        extra["rank_one_512x256"] = r
        wl["rank_one_512x256_uv"] = dict(ms=r["ms"], sigma_per_s=r["sigma_per_s"], sweeps=r["info"][1:3])
        note("rectangular layers done")
    if sel("strided"):
        # stride-2 layers as crystals (s*s input points per coarse cell)
        for name, Ls, s, Ws in workloads.resnet18_downsampling():
            r = run_strided(Ls, s, Ws, dev, reps * 3, 1)
            key = "strided_" + name
            extra[key] = r
            c = r["crystal"]
            wl[key + "_64to128_32x32_s2_uv"] = dict(
                ms=r["ms"], sigma_per_s=r["sigma_per_s"], sweeps=r["info"][1:3],
                crystal_layer=[c.c_out, c.c_in, c.kh, c.kw, c.n, c.m])
        note("strided layers done")
    if sel("split"):
        # transformation vs SVD (the paper's Table III), and the fused path
        Lp, Wp = workloads.paper_scale(1024)
        sp = bench_split(dev, reps, Lp, Wp, False)
        # Table III, LFA at n = 1024: transformation 1.28 s, SVD 31.74 s (Xeon Gold 6242, NumPy)
        sp.update(paper_transform_s=1.28, paper_svd_s=31.74, paper_transform_share=1.28 / (1.28 + 31.74))
        wl["split_paper_scale_c16_n1024"] = sp
        wl["split_64x64_uv"] = bench_split(dev, reps, L, W, True)
        note("assembly / SVD split done")
    if sel("stack"):
        st = bench_stack(dev, reps)
        extra["stack"] = st
        wl["resnet18_stack_sigma_grad"] = {
            "layers": 12, "loss": "sum of top-8 sigma per layer",
            "plain_layers_per_s": st["plain_layers_per_s"], "batched_layers_per_s": st["batched_layers_per_s"],
            "plain_ms": st["plain_ms"], "batched_ms": st["batched_ms"],
            "batched": "HIP graph: persistent SVD keeping U of every symbol, top-8, one-sided adjoint",
            "plain": "eager: lfa_svd per layer keeping U, lfa_topk, lfa_adjoint_onesided",
            "batched_uv_graph_ms": st["batched_uv_graph_ms"],
            "batched_sigma_only_graph_ms": st["batched_sigma_only_ms"],
            "plain_sigma_only_recompute_ms": st["plain_sigma_only_recompute_ms"],
            "autotuned": st["tuned"],
            "batched_roofline": st["roofline"],
            "timed": "the faster of the default and the autotuned plan for each path",
            "speedup_batched_vs_plain": st["batched_layers_per_s"] / st["plain_layers_per_s"]}
        note("ResNet-18 stack done")
    if sel("large"):
        L5, W5, _ = workloads.large_grid_7x7()
        for asm in (None, "bf16x2", "bf16x3"):
            r = run_layer(L5, W5, dev, False, reps, 1, asm=asm)
            key = "large_grid_7x7_" + (asm or "fp32")
            extra[key] = r
            wl[key] = dict(ms=r["ms"], sigma_per_s=r["sigma_per_s"], sweeps=r["info"][1:3], vectors=False)
            note(f"large grid {key} done")
    if sel("assembly"):
        for asm in ("valu", "mfma", "bf16x3"):
            a = bench_assembly(dev, 5, asm)
            extra["assembly_" + asm] = a
            wl["assembly_224x224_7x7_" + asm] = dict(ms=a["ms"], hbm_gbs=a["gbs"],
                                                     frac_of_hbm_peak=a["gbs"] / PEAK_HBM_GBS)
        note("assembly kernels done")
    if sel("paper"):
        # the paper's own runtime study (Tables II, III): c = 16, 3x3, sigma only
        for n in (1024, 16384):
            Lp, Wp = workloads.paper_scale(n)
            r = run_layer(Lp, Wp, dev, False, 2 if n > 4096 else reps, 1)
            key = f"paper_scale_c16_n{n}"
            extra[key] = r
            wl[key] = dict(ms=r["ms"], sigma_per_s=r["sigma_per_s"], sweeps=r["info"][1:3], vectors=False,
                           paper_cpu_seconds=PAPER_TABLE2_SECONDS[n],
                           paper_hardware="Xeon Gold 6242, 16 cores, NumPy (Table II)",
                           speedup_vs_paper=PAPER_TABLE2_SECONDS[n] / (r["ms"] * 1e-3))
            note(f"paper scale n={n} done")
    if not args.quick:
        line["workloads"] = wl
    if not args.no_cpu:
        note("oracle legs (CPU) start")
        cb, errors = cpu_leg(head, extra)
        line["cpu_baseline"] = cb
        line["sigma_error_vs_oracle"] = errors
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
