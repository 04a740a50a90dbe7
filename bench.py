"""Benchmark of the Brand-update K-factor path on one MI355X.

Workload (the headline shape): a 24-layer MLP-like stack with both K-factors
of every layer at width d = 4096 (48 independent factor states), truncation
rank r = 256, batch width n = 256, rho = 0.95, lambda = 0.01, in the
BF16-mixed precision form.  One step is one pass of the whole hot path over
one synthetic batch per state: a grouped Brand update of all 48 states
(truncate, projection, residual, CholeskyQR, core eigensolve, rotation) plus a
grouped two-sided preconditioning of all 24 layer gradients.  All inputs are
generated on the device before the timed region.

Reported: B-updates/s over the timed steps (the 24 preconditionings are done
inside the same steps), the FP32-plain form's B-updates/s (one state at a
time, no grouping) beside it, per-step latency p50/p99, the roofline of the
dominant kernel from HIP events recorded live around every stage, and the
FP64 CPU oracle timed on a bounded sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "hbm_gbs": 8000.0}
LAYERS, D, R, N_BATCH, RHO, LAM = 24, 4096, 256, 256, 0.95, 0.01


def _gen_batches(torch, dev, states, n, d, seed, dtype):
    """Seeded synthetic batches on the device: ReLU(z k^-1) for A, z k^-0.7 for Gamma."""
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    k = torch.arange(1, d + 1, device=dev, dtype=torch.float32)
    out = []
    for i in range(states):
        z = torch.randn(n, d, generator=g, device=dev)
        x = torch.relu(z * k ** -1.0) if i % 2 == 0 else z * k ** -0.7
        out.append(x.to(dtype).contiguous())
    return out


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def cpu_baseline(budget_s: float = 8.0):
    """The FP64 oracle timed on the host cores at the headline shape: Oracle-B (the
    structured Brand update, Algorithm 3) and Oracle-D (the dense definition: the
    d x d B-process iterate and a full eigendecomposition per update), each with
    the BLAS pool on all host cores and on one core; median over the samples that
    fit the time budget (at least one each)."""
    import numpy as np
    import oracle
    from paper_2210_08494_amd import synth
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=os.cpu_count())
    except Exception:
        threadpool_limits, threads = None, os.cpu_count()

    def warm(make):
        f = make()
        for k in range(2):  # bring the state to r + n = 512 modes (untimed, all cores)
            f.update(synth.batch_for(6, k, "A", N_BATCH, D).T)
        return f

    def run(f, budget, max_samples, k0):
        times, k = [], k0
        t_all = time.perf_counter()
        while len(times) < max_samples and (not times or time.perf_counter() - t_all < budget):
            M = synth.batch_for(6, k, "A", N_BATCH, D).T
            t0 = time.perf_counter()
            f.update(M)
            times.append(time.perf_counter() - t0)
            k += 1
        return float(np.median(times)), len(times)

    res = {}
    for name, make, budget, cap in (("oracle_b", lambda: oracle.BrandFactor(D, R, RHO), budget_s, 100),
                                    ("oracle_d", lambda: oracle.DenseFactor(D, R, RHO), 0.0, 1)):
        f = warm(make)
        for cores in ("all", "1"):
            if cores == "1" and threadpool_limits is None:
                continue
            if cores == "1":
                with threadpool_limits(limits=1):
                    med, cnt = run(f, budget, cap, 200)
            else:
                med, cnt = run(f, budget, cap, 2)
            res[f"{name}_{cores}"] = {"s_per_update": round(med, 4), "b_updates_per_s": round(1.0 / med, 4),
                                      "samples": cnt, "threads": int(threads) if cores == "all" else 1}
    main = res["oracle_b_all"]
    return {"value": main["b_updates_per_s"], "unit": "B-updates/s", "cores": main["threads"], "kind": "oracle",
            "sample": f"{main['samples']} structured FP64 Brand updates (oracle/brand.py, Householder QR + "
                      f"eigh of the {R + N_BATCH}-wide core) at d={D} r={R} n={N_BATCH} on the host, median "
                      f"{main['s_per_update']:.3f} s each; beside it the dense definition (oracle/bprocess.py, "
                      f"eigh of the {D}x{D} iterate) and both on one core",
            "legs": res}


def _cu_masked_streams(torch, dev, n_pre):
    """Two streams on disjoint sets of CUs (hipExtStreamCreateWithCUMask, default
    priority): the first ncu - n_pre CUs for the update, the last n_pre for the
    preconditioning.  None when the runtime refuses the masks."""
    import ctypes
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    if not 0 < n_pre < ncu:
        return None
    hip = ctypes.CDLL("libamdhip64.so")
    words = (ncu + 31) // 32
    out = []
    for cus in (range(0, ncu - n_pre), range(ncu - n_pre, ncu)):
        mask = (ctypes.c_uint32 * words)()
        for c in cus:
            mask[c // 32] |= 1 << (c % 32)
        h = ctypes.c_void_p()
        if hip.hipExtStreamCreateWithCUMask(ctypes.byref(h), ctypes.c_uint32(words), mask) != 0:
            return None
        out.append(torch.cuda.ExternalStream(h.value, device=dev))
    return out[0], out[1], ncu - n_pre, n_pre


def _measured_traffic(kfb, kname):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, only when it was taken on this exact library build."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"{kname}_d4096_r256_n256_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    build = kfb.load().kfb_build_info().decode()
    if vals.get("library") != build or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


class _BatchPool:
    """Distinct pre-generated batches in HBM, handed out in order: every update
    request of a serving run gets a batch no state has seen (the pool wraps
    around only if a run needs more than it holds)."""

    def __init__(self, torch, dev, count, n, d, seed, dtype):
        self.sets = {}
        for s_i, side in enumerate(("A", "G")):
            g = torch.Generator(device=dev)
            g.manual_seed(seed + s_i)
            k = torch.arange(1, d + 1, device=dev, dtype=torch.float32)
            out = []
            for _ in range(count):
                z = torch.randn(n, d, generator=g, device=dev)
                x = torch.relu(z * k ** -1.0) if side == "A" else z * k ** -0.7
                out.append(x.to(dtype).contiguous())
            self.sets[side] = out
        self.next = {"A": 0, "G": 0}

    def take(self, side):
        i = self.next[side]
        self.next[side] = i + 1
        b = self.sets[side]
        return b[i % len(b)]


def _serve_stats(serve, srv, wall, done):
    lat_ms = [1e3 * (r.t_done - r.t_arrival) for r in done]
    upd = sum(1 for r in done if isinstance(r, serve.UpdateRequest))
    return {"requests": len(done), "updates": upd, "preconditionings": len(done) - upd,
            "p50_ms": round(serve.percentile(lat_ms, 50), 3), "p99_ms": round(serve.percentile(lat_ms, 99), 3),
            "achieved_req_per_s": round(len(done) / wall, 1), "b_updates_per_s": round(upd / wall, 1),
            "mean_group": round(srv.stats.grouped_problems / max(srv.stats.groups, 1), 2),
            "mean_update_group": round(srv.stats.update_problems / max(srv.stats.update_groups, 1), 2)}


def serve_leg(torch, kfb, dev, args, prec, nreq, grouped=True):
    """Open-loop Poisson serving at the headline shape (24 layers, 48 states at
    d=4096, r=256, n=256): 70% updates (uniform over layer and factor), 30%
    preconditionings (uniform layer), a fresh batch for every update.  First at
    2000 requests/s offered (above the capacity of either form: the achieved rate
    is the form's saturation), then at half of that measured saturation.  The
    mixed form runs with continuous batching (grouped launches, up to 48 per
    group, four streams); the FP32-plain form one request at a time on one
    stream (no grouping)."""
    from paper_2210_08494_amd import serve
    L = args.layers
    layers = [(D, D, R, R)] * L
    mdt = torch.bfloat16 if prec == kfb.KFB_BF16_MIXED else torch.float32
    srv = serve.Server(layers, n_max=N_BATCH, rho=RHO, prec=prec, streams=4 if grouped else 1,
                       byte_budget=24 << 30, max_group=48 if grouped else 1,
                       max_inflight=None if grouped else 1)
    # two runs of nreq requests, 70% of them updates, half on each side: ~0.7 nreq per side
    pool = _BatchPool(torch, dev, int(0.75 * nreq) + 2 * L + 64, N_BATCH, D, seed=5000 + prec, dtype=mdt)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    grads = [torch.randn(D, D, generator=gen, device=dev) for _ in range(L)]
    outs = [torch.empty(D, D, device=dev) for _ in range(L)]
    torch.cuda.synchronize()
    for j in range(2):  # bring every state to r + n modes
        for l in range(L):
            for side in ("A", "G"):
                srv.submit(serve.UpdateRequest(l, side, pool.take(side)))
    srv.drain()
    torch.cuda.synchronize()

    def make(i, rng):
        l = int(rng.integers(L))
        if rng.random() < 0.7:
            side = "A" if rng.random() < 0.5 else "G"
            return serve.UpdateRequest(l, side, pool.take(side))
        return serve.PrecondRequest(l, grads[l], outs[l], LAM, LAM)

    res = {"mode": "continuous batching, grouped launches" if grouped else "one request at a time, no grouping"}
    srv.stats = serve.ServerStats()
    prog = lambda i, c, t: _progress(f"serving prec={prec}: {i} submitted, {c} done, {t:.0f} s")
    wall, done = serve.poisson_run(srv, make, 2000.0, nreq, seed=2000 + prec, timeout_s=600.0, progress=prog)
    res["2000_req_per_s"] = _serve_stats(serve, srv, wall, done)
    _progress(f"serving prec={prec} at 2000 req/s: {res['2000_req_per_s']}")
    sat = res["2000_req_per_s"]["achieved_req_per_s"]
    half = max(0.5 * sat, 1.0)
    srv.stats = serve.ServerStats()
    wall, done = serve.poisson_run(srv, make, half, nreq, seed=1000 + prec, timeout_s=900.0, progress=prog)
    res["half_saturation"] = dict(_serve_stats(serve, srv, wall, done), offered_req_per_s=round(half, 1))
    res["pool_batches"] = len(pool.sets["A"]) + len(pool.sets["G"])
    res["batches_used"] = pool.next["A"] + pool.next["G"]
    del pool, srv
    return res


def serve_mixed_leg(torch, kfb, dev, args):
    """Open-loop Poisson serving of a 24-layer MLP-shaped stream at uneven widths and
    ranks: widths w_0..w_24 drawn from {512, ..., 8192} (layer l: d_in = w_l,
    d_out = w_{l+1}), r per factor drawn from {64, ..., 512} and clamped to d - 256,
    n per update request drawn from {64, 128, 256}; 70% updates (uniform over layer
    and factor), 30% preconditionings (uniform layer), BF16-mixed.  Updates of every
    factor that keeps the same number of modes share a group whatever its width and
    batch width (kfb_brand_update_grouped pads them on the device)."""
    import numpy as np
    from paper_2210_08494_amd import serve
    L = args.layers
    rng = np.random.default_rng(24)
    widths = [int(x) for x in rng.choice([512, 1024, 2048, 4096, 8192], size=L + 1)]
    ranks = [int(x) for x in rng.choice([64, 128, 256, 512], size=L)]
    nmax = 256
    layers = [(widths[l], widths[l + 1], min(ranks[l], widths[l] - nmax), min(ranks[l], widths[l + 1] - nmax))
              for l in range(L)]
    srv = serve.Server(layers, n_max=nmax, rho=RHO, prec=kfb.KFB_BF16_MIXED, streams=4,
                       byte_budget=24 << 30, max_group=48, pad_updates=True, max_inflight=args.uneven_inflight)
    # per factor a ring of distinct 256-sample batches; a request of width n takes
    # the first n samples of the next one
    ring = 16
    pool, nxt = {}, {}
    for l, (d_in, d_out, _, _) in enumerate(layers):
        for s_i, (side, d) in enumerate((("A", d_in), ("G", d_out))):
            pool[(l, side)] = [b for j, b in enumerate(_gen_batches(torch, dev, 2 * ring, nmax, d,
                                                                    seed=7000 + 2 * l + s_i,
                                                                    dtype=torch.bfloat16)) if j % 2 == s_i]
            nxt[(l, side)] = 0

    def take(l, side, n):
        i = nxt[(l, side)]
        nxt[(l, side)] = i + 1
        return pool[(l, side)][i % ring][:n]
    gen = torch.Generator(device=dev)
    gen.manual_seed(12)
    grads = [torch.randn(d_out, d_in, generator=gen, device=dev) for (d_in, d_out, _, _) in layers]
    outs = [torch.empty_like(g) for g in grads]
    torch.cuda.synchronize()
    for j in range(2):  # every state to r + n modes
        for l in range(L):
            for side in ("A", "G"):
                srv.submit(serve.UpdateRequest(l, side, take(l, side, nmax)))
    srv.drain()
    torch.cuda.synchronize()

    def make(i, rng):
        l = int(rng.integers(L))
        if rng.random() < 0.7:
            side = "A" if rng.random() < 0.5 else "G"
            n = int(rng.choice([64, 128, 256]))
            return serve.UpdateRequest(l, side, take(l, side, n))
        return serve.PrecondRequest(l, grads[l], outs[l], LAM, LAM)

    res = {"widths": widths, "ranks": [(a, g) for (_, _, a, g) in layers]}
    # an offered rate far above capacity (throughput) and one below it (latency)
    for rate, nreq in ((2000.0, args.serve_requests_uneven), (150.0, max(args.serve_requests_uneven // 2, 1))):
        srv.stats = serve.ServerStats()
        wall, done = serve.poisson_run(srv, make, rate, nreq, seed=2024 + int(rate))
        lat_ms = [1e3 * (r.t_done - r.t_arrival) for r in done]
        upd = sum(1 for r in done if isinstance(r, serve.UpdateRequest))
        res[f"{int(rate)}_req_per_s"] = {
            "requests": len(done), "updates": upd, "preconditionings": len(done) - upd,
            "p50_ms": round(serve.percentile(lat_ms, 50), 3), "p99_ms": round(serve.percentile(lat_ms, 99), 3),
            "achieved_req_per_s": round(len(done) / wall, 1), "b_updates_per_s": round(upd / wall, 1),
            "mean_group": round(srv.stats.grouped_problems / max(srv.stats.groups, 1), 2),
            "mean_update_group": round(srv.stats.update_problems / max(srv.stats.update_groups, 1), 2)}
        _progress(f"uneven serving at {rate} req/s: {res[f'{int(rate)}_req_per_s']}")
    return res


def _progress(msg):
    # one line per finished leg on stderr (stdout carries only the JSON line)
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--layers", type=int, default=LAYERS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-updates", type=int, default=6)
    ap.add_argument("--graph-steps", type=int, default=20)
    ap.add_argument("--fp32-grouped-steps", type=int, default=5)
    ap.add_argument("--sequential-steps", type=int, default=5)
    ap.add_argument("--one-stream", action="store_true",
                    help="time the step with its two calls in sequence on one stream")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-requests-fp32", type=int, default=2000)
    ap.add_argument("--serve-requests-uneven", type=int, default=2000)
    ap.add_argument("--uneven-inflight", type=int, default=8, help="groups in flight in the uneven serving leg")
    ap.add_argument("--cu-split", default="auto",
                    help="CUs of the preconditioning's stream in the two-stream step ('auto': what the "
                         "update's eigensolver rounds leave at two workgroups per CU; 'off': unmasked streams)")
    ap.add_argument("--jacobi-config", default="",
                    help="install this eigensolver configuration instead of autotuning (e.g. 0x320: "
                         "FP32 iteration + FP64 refinement, 0x120: FP64 iteration)")
    ap.add_argument("--gemm-tile", type=int, default=0,
                    help="install this output tile for the preconditioner's products instead of autotuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (factor states "
              "are independent: a multi-GPU run would place whole layers per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2210_08494_amd import kfb
    kfb.load()
    dev = torch.device("cuda:0")
    L = args.layers
    S = 2 * L
    MIX = kfb.KFB_BF16_MIXED

    # ---- autotune the core eigensolver's configuration for this bucket (untimed)
    from paper_2210_08494_amd import tune
    if args.jacobi_config:
        best_bw, tune_ms = int(args.jacobi_config, 0), {}
        kfb.tune_set_jacobi(MIX, R + N_BATCH, best_bw)
    else:
        best_bw, tune_ms = tune.tune_jacobi(MIX, D, R, N_BATCH, count=S, reps=2, device=dev)
    _progress(f"autotune done: {best_bw}")

    # ---- states: even index = A factor (d_in), odd = Gamma factor (d_out) of a layer
    states = [kfb.Factor(D, R, N_BATCH, RHO, MIX, device=dev) for _ in range(S)]
    # a fresh synthetic batch for every state at every step and a fresh gradient for
    # every layer at every step, all generated into HBM before the timed region (no
    # batch repeats: an absorbed batch lies in span(U) and would degenerate the core)
    nsets = 1 + args.warmup + args.steps
    batches = [_gen_batches(torch, dev, S, N_BATCH, D, seed=1000 + j, dtype=torch.bfloat16) for j in range(nsets)]
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    Gsets = [[torch.randn(D, D, generator=gen, device=dev) for _ in range(L)] for _ in range(nsets)]
    Ss = [torch.empty(D, D, device=dev) for _ in range(L)]
    ws_u, ws_p = kfb.Workspace(dev), kfb.Workspace(dev)
    fa = states[0::2]
    fg = states[1::2]
    lam = [LAM] * L

    def step_seq(j):
        kfb.update_batched(states, batches[j], ws_u)
        kfb.precondition_batched(fg, fa, Gsets[j], Ss, lam, lam, 0, ws_p)

    # The timed step runs its two calls on two streams at once: the
    # preconditioning reads the factors the previous update left in the front
    # buffers while this step's update writes the back buffers (the states are
    # double-buffered for this).  The preconditioning is enqueued first (the
    # library takes the front buffers at enqueue) and waits for the previous
    # update; the update waits for the previous preconditioning, which read the
    # buffers it is about to write.  The two streams run on disjoint CUs
    # (--cu-split): the update keeps as many as its eigensolver rounds fill at
    # two workgroups per CU (48 cores x 8 block pairs = 384 workgroups -> 192
    # CUs), the preconditioning's products take the rest, so they never hold CUs
    # that a round's workgroups wait for (each round lasts as long as its
    # slowest workgroup).
    streams = None
    if args.cu_split != "off" and not args.one_stream:
        pairs = (R + N_BATCH + 63) // 64   # block pairs of 32-column blocks per round
        n_pre = (torch.cuda.get_device_properties(dev).multi_processor_count - S * pairs // 2
                 if args.cu_split == "auto" else int(args.cu_split))
        streams = _cu_masked_streams(torch, dev, n_pre)
        _progress(f"CU-masked streams: {streams[2:] if streams else None}")
    if streams:
        s_upd, s_pre, cus_upd, cus_pre = streams
    else:
        s_upd, s_pre, cus_upd, cus_pre = torch.cuda.current_stream(), torch.cuda.Stream(device=dev), None, None
    pipe = {"u": None, "p": None}

    def step(j):
        if args.one_stream:   # the sequential form (profiling runs: per-kernel durations without overlap)
            step_seq(j)
            return
        with torch.cuda.stream(s_pre):
            if pipe["u"] is not None:
                s_pre.wait_event(pipe["u"])
            kfb.precondition_batched(fg, fa, Gsets[j], Ss, lam, lam, 0, ws_p)
            ep = torch.cuda.Event()
            ep.record(s_pre)
        with torch.cuda.stream(s_upd):
            if pipe["p"] is not None:
                s_upd.wait_event(pipe["p"])
            kfb.update_batched(states, batches[j], ws_u)
            eu = torch.cuda.Event()
            eu.record(s_upd)
        pipe["u"], pipe["p"] = eu, ep

    # first update takes every state from empty to n modes; warmup reaches r + n
    kfb.update_batched(states, batches[0], ws_u)
    for j in range(args.warmup):
        step(1 + j)
    torch.cuda.synchronize()
    # ---- autotune the output tile of the preconditioner's BF16 products (untimed)
    Ncore = R + N_BATCH
    if args.gemm_tile:
        tile_best, tile_ms = args.gemm_tile, {}
        for (m, n, k) in tune.precond_product_shapes(D, D, Ncore, Ncore):
            kfb.tune_set_gemm(m, n, k, tile_best)
    else:
        # timed where the step runs it: on the preconditioning's stream (its CU share)
        with torch.cuda.stream(s_pre):
            tile_best, tile_ms = tune.tune_gemm_tiles(
                lambda: kfb.precondition_batched(fg, fa, Gsets[0], Ss, lam, lam, 0, ws_p),
                tune.precond_product_shapes(D, D, Ncore, Ncore), reps=3)
    _progress(f"gemm tile autotune done: {tile_best} {tile_ms}")

    # ---- timed region (stage events recorded live on the same stream)
    kfb.profile_enable(True)
    kfb.profile_report(reset=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s_rec = torch.cuda.current_stream() if args.one_stream else s_upd
    ev[0].record(s_rec)
    for j in range(args.steps):
        step(1 + args.warmup + j)
        ev[j + 1].record(s_rec)
    s_upd.wait_stream(s_pre)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = kfb.profile_report(reset=True)
    kfb.profile_enable(False)
    step_ms = [ev[j].elapsed_time(ev[j + 1]) for j in range(args.steps)]
    status = [f.status() for f in states]
    if streams:
        # a CU-masked stream holds a hardware queue of its own; give both back before
        # the serving legs, whose streams share the process's few queues
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        for st in (s_upd, s_pre):
            hip.hipStreamDestroy(ctypes.c_void_p(st.cuda_stream))
        s_upd = s_pre = None

    bups = S * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    _progress(f"timed region: {bups:.1f} B-updates/s, {ms_per_step:.3f} ms per step")

    # ---- roofline of the dominant kernel (core eigensolver rounds)
    Ncore = R + N_BATCH
    # the eigensolve of a core is the main iteration plus the pre-rotation of its
    # new-direction block (both launch the same round kernel)
    jac = dict(prof.get("jacobi", {"ms": float("nan"), "launches": 1, "calls": 1}))
    jpre = prof.get("jacobi_pre")
    if jpre:
        jac["ms"] += jpre["ms"]
        jac["launches"] += jpre["launches"]
    calls = max(prof.get("jacobi", {"calls": 1})["calls"], 1)
    launches_per_call = jac["launches"] / calls
    avg_launch_ms = jac["ms"] / max(jac["launches"], 1)
    flops_per_call = S * 9.0 * Ncore ** 3  # textbook symmetric EVD count per core
    flops_per_launch = flops_per_call / launches_per_call
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    cfg = kfb.tune_get_jacobi(MIX, Ncore)[0]
    refined = bool(cfg & kfb.KFB_JAC_REFINE)
    peak = PEAK["fp32"] if refined else PEAK["fp64"]
    if cfg & kfb.KFB_JAC_STREAMED:
        kname = {16: "jacobi_s_kernel", 32: "jacobi_g_kernel"}[cfg & 0xFF]
        if refined:
            kdesc = (f"{kname}<float> (block one-sided Jacobi round on FP32 MFMA, 64-column panels streamed "
                     f"from HBM; the eigenpairs then refined in FP64)")
            tname = f"{kname}_fp32"
        else:
            kdesc = f"{kname}<double> (block one-sided Jacobi round, FP64, {2 * (cfg & 0xFF)}-column panels streamed from HBM)"
            tname = kname
    else:
        kdesc = f"jacobi_kernel<double,{cfg}> (block one-sided Jacobi round, FP64, panel in LDS)"
        tname = "jacobi_kernel"
    traffic = _measured_traffic(kfb, tname)
    # the whole eigensolve of a call (iteration rounds, FP64 refinement, finalize)
    # in the same unit, against the FP64 peak: the result the stage delivers is FP64
    eig_ms = sum(prof[k]["ms"] for k in ("jacobi", "jacobi_pre", "refine", "finalize") if k in prof) / calls
    eig_tf = flops_per_call / (eig_ms * 1e-3) / 1e12
    roofline = {"kernel": kdesc,
                "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "per_launch": {"algorithmic_flops": flops_per_launch, "avg_ms": avg_launch_ms,
                               "launches_per_update_call": launches_per_call,
                               "unit_work": "9*(r+n)^3 flops per core eigensolve (main iteration and the "
                                            "pre-rotation of the new-direction block), 48 cores per call"},
                "eigensolve_stage": {"ms_per_call": round(eig_ms, 4), "achieved": round(eig_tf, 3),
                                     "peak": PEAK["fp64"], "frac": round(eig_tf / PEAK["fp64"], 4),
                                     "note": "9*(r+n)^3 per core over the whole eigensolve stage (rounds, "
                                             "FP64 refinement, finalize) against the FP64 peak"}}

    # other stages, algorithmic work per call
    def _rate(stage, flops):
        st = prof.get(stage)
        if not st or st["calls"] == 0:
            return None
        ms = st["ms"] / st["calls"]
        return {"ms_per_call": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 3)}

    r, n, N = R, N_BATCH, Ncore
    stages = {
        "proj": _rate("proj", S * (2 * 2.0 * D * r * n + 2 * 2.0 * D * r * n)),
        "cholqr": _rate("cholqr", S * 2 * (2.0 * D * n * n + 2.0 * D * n * n)),
        "core": _rate("core", S * 2.0 * N * N),
        "jacobi": _rate("jacobi", S * 9.0 * N ** 3),
        "jacobi_pre": _rate("jacobi_pre", S * 9.0 * n ** 3),
        "refine": _rate("refine", S * 4 * 2.0 * N ** 3),
        "finalize": _rate("finalize", S * 2.0 * N * N),
        "rotate": _rate("rotate", S * 2.0 * D * N * N),
        "pre_coef_T1_T2_T3": _rate("pre_coef_T1_T2_T3", L * (2 * 2.0 * N * D * D + 2.0 * N * N * D)),
        "pre_scale_X2": _rate("pre_scale_X2", L * 2.0 * D * N * N),
        "pre_S": _rate("pre_S", L * 2.0 * D * D * 2 * N),
    }

    # ---- the same step with its two calls one after the other on one stream
    sequential = None
    if args.sequential_steps > 0:
        seq_sets = [_gen_batches(torch, dev, S, N_BATCH, D, seed=2000 + j, dtype=torch.bfloat16)
                    for j in range(args.sequential_steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(args.sequential_steps):
            kfb.update_batched(states, seq_sets[j], ws_u)
            kfb.precondition_batched(fg, fa, Gsets[j % nsets], Ss, lam, lam, 0, ws_p)
        torch.cuda.synchronize()
        sw = time.perf_counter() - t0
        sequential = {"value": round(S * args.sequential_steps / sw, 2), "unit": "B-updates/s",
                      "ms_per_step": round(1e3 * sw / args.sequential_steps, 3), "steps": args.sequential_steps,
                      "note": "the same step with the update and the preconditioning in sequence on one stream"}
        del seq_sets
        _progress(f"sequential step: {sequential}")

    # ---- the same step replayed from a HIP graph: two consecutive steps captured
    # (every state's front and back buffers trade roles twice and end as they
    # began) over two batch slots; before each replay the next two fresh batch
    # sets are copied into the slots (device-to-device, inside the timed region:
    # ~200 MB per replay), so no replay re-feeds a batch; the library launches
    # only kernels on the caller's stream, so the whole step is capturable
    graph_replay = None
    if args.graph_steps > 0:
        reps = max(args.graph_steps // 2, 1)
        gsets = [_gen_batches(torch, dev, S, N_BATCH, D, seed=3000 + j, dtype=torch.bfloat16)
                 for j in range(2 * reps + 2)]
        slots = [[torch.empty_like(b) for b in batches[0]] for _ in range(2)]

        def gstep(q):   # the sequential form of the step (one stream)
            kfb.update_batched(states, slots[q], ws_u)
            kfb.precondition_batched(fg, fa, Gsets[q], Ss, lam, lam, 0, ws_p)

        def refill(j):
            for q in range(2):
                for dst, src in zip(slots[q], gsets[2 * j + q]):
                    dst.copy_(src)
        torch.cuda.synchronize()
        refill(reps)   # capture-time contents (the capture performs no work)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gstep(0)
            gstep(1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(reps):
            refill(j)
            graph.replay()
        torch.cuda.synchronize()
        gwall = time.perf_counter() - t0
        graph_replay = {"value": round(S * 2 * reps / gwall, 2), "unit": "B-updates/s",
                        "ms_per_step": round(1e3 * gwall / (2 * reps), 3), "steps": 2 * reps,
                        "note": "the timed step (grouped updates + grouped preconditioning) captured "
                                "in one HIP graph and replayed; fresh batches copied into the graph's "
                                "input slots before each replay (copies timed)"}
        del graph, gsets, slots

    _progress("timed steps and graph replay done")
    # ---- FP32 plain form: one state at a time, no grouping, fresh batch per update
    f32 = [kfb.Factor(D, R, N_BATCH, RHO, kfb.KFB_FP32, device=dev) for _ in range(2)]
    b32 = _gen_batches(torch, dev, 4 + args.fp32_updates, N_BATCH, D, seed=99, dtype=torch.float32)
    for j in range(2):
        for i, f in enumerate(f32):
            f.update(b32[2 * j + i])
    torch.cuda.synchronize()
    lat32 = []
    for i in range(args.fp32_updates):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        f32[i % 2].update(b32[4 + i])
        e1.record()
        torch.cuda.synchronize()
        lat32.append(e0.elapsed_time(e1))
    fp32_plain = None
    if lat32:
        fp32_plain = {"value": round(1e3 / (sum(lat32) / len(lat32)), 2), "unit": "B-updates/s",
                      "ms_per_update_p50": round(_percentile(lat32, 50), 3), "states": 2,
                      "mode": "one update at a time, no grouping"}
    del f32, b32

    # ---- FP32 form grouped like the headline (48 states, one grouped update and
    # 24 grouped preconditionings per step, fresh inputs): isolates the precision
    # form's effect from the grouping's
    fp32_grouped = None
    if args.fp32_grouped_steps > 0:
        st32 = [kfb.Factor(D, R, N_BATCH, RHO, kfb.KFB_FP32, device=dev) for _ in range(S)]
        nq = 3 + args.fp32_grouped_steps
        bq = [_gen_batches(torch, dev, S, N_BATCH, D, seed=5000 + j, dtype=torch.float32) for j in range(nq)]
        fa32, fg32 = st32[0::2], st32[1::2]
        wsu32, wsp32 = kfb.Workspace(dev), kfb.Workspace(dev)

        def step32(j):
            kfb.update_batched(st32, bq[j], wsu32)
            kfb.precondition_batched(fg32, fa32, Gsets[j % nsets], Ss, lam, lam, 0, wsp32)
        kfb.update_batched(st32, bq[0], wsu32)
        step32(1)
        step32(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(args.fp32_grouped_steps):
            step32(3 + j)
        torch.cuda.synchronize()
        w32 = time.perf_counter() - t0
        fp32_grouped = {"value": round(S * args.fp32_grouped_steps / w32, 2), "unit": "B-updates/s",
                        "ms_per_step": round(1e3 * w32 / args.fp32_grouped_steps, 3),
                        "steps": args.fp32_grouped_steps,
                        "mode": f"FP32 form, the headline step: grouped update of {S} states + grouped "
                                f"preconditioning of {L} layers, fresh batches"}
        del st32, bq, wsu32, wsp32

    _progress("fp32 leg done")
    # ---- factored (linear-cost) application, Algorithm 8: the gradient of each
    # layer given as G_k A_k^T by the step's own batches (grouped over the layers)
    Gks = [batches[0][2 * l + 1] for l in range(L)]
    Aks = [batches[0][2 * l] for l in range(L)]
    ws_f = kfb.Workspace(dev)
    kfb.precondition_factored_batched(fg, fa, Gks, Aks, Ss, lam, lam, 0, ws_f)
    torch.cuda.synchronize()
    fac_ms = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        kfb.precondition_factored_batched(fg, fa, Gks, Aks, Ss, lam, lam, 0, ws_f)
        e1.record()
        torch.cuda.synchronize()
        fac_ms.append(e0.elapsed_time(e1))
    fac_call = _percentile(fac_ms, 50)
    # the two-sided call on the same inputs, alone on the whole GPU (its stage times
    # in the timed step are taken on the preconditioning's share of the CUs)
    two_ms = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        kfb.precondition_batched(fg, fa, Gsets[0], Ss, lam, lam, 0, ws_p)
        e1.record()
        torch.cuda.synchronize()
        two_ms.append(e0.elapsed_time(e1))
    two_sided = _percentile(two_ms, 50)
    fac_flops = L * (2 * 4.0 * N * D * n + 2.0 * D * D * n)
    factored = {"ms_per_call": round(fac_call, 3), "layers": L,
                "ms_per_layer": round(fac_call / L, 4),
                "two_sided_ms_per_layer": round(two_sided / L, 4),
                "speedup_vs_two_sided": round(two_sided / fac_call, 2),
                "tflops": round(fac_flops / (fac_call * 1e-3) / 1e12, 2),
                "s_write_gbs": round(L * 4.0 * D * D / (fac_call * 1e-3) / 1e9, 1),
                "unit_work": "per layer 8*N*d*n (both sides) + 2*d^2*n (S = Y_G Y_A^T) flops; S written once (FP32)"}

    _progress("factored leg done")
    # ---- B-R-KFAC pieces at the same shape: one dense EA-factor step and one
    # randomized-SVD overwrite (oversampling 16, two power iterations)
    fbr = kfb.Factor(D, R, N_BATCH, RHO, MIX, device=dev)
    Xd = kfb.dense_factor(fbr, device=dev)
    kfb.dense_update(fbr, Xd, batches[0][0], first=True)
    for j in range(2):
        fbr.update(batches[j][0])
        kfb.dense_update(fbr, Xd, batches[j][0], first=False)
    gsk = torch.Generator(device=dev)
    gsk.manual_seed(13)
    Om = torch.randn(R + 16, D, generator=gsk, device=dev)
    kfb.rsvd_overwrite(fbr, Xd, Om, 16, 2)
    torch.cuda.synchronize()

    def _time(fn, reps):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return _percentile(ts, 50)
    dense_ms = _time(lambda: kfb.dense_update(fbr, Xd, batches[1][0], first=False), 5)
    rsvd_ms = _time(lambda: kfb.rsvd_overwrite(fbr, Xd, Om, 16, 2), 3)
    brkfac = {"dense_update_ms": round(dense_ms, 3),
              "dense_update_tflops": round(2.0 * D * D * N_BATCH / (dense_ms * 1e-3) / 1e12, 1),
              "rsvd_overwrite_ms": round(rsvd_ms, 3),
              "rsvd_tflops": round(6 * 2.0 * D * D * (R + 16) / (rsvd_ms * 1e-3) / 1e12, 1),
              "config": f"one factor, d={D}, r={R}, l={R + 16}, 2 power iterations; dense factor FP32",
              "unit_work": "dense step 2*d^2*n flops; RSVD 6 products 2*d^2*l (sketch, 2 x 2 power, final)"}
    del Xd

    _progress("brkfac leg done")
    # ---- single mixed update latency (no grouping), for the latency columns
    lat1 = []
    b1 = _gen_batches(torch, dev, 6, N_BATCH, D, seed=4000, dtype=torch.bfloat16)
    for i in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        states[i].update(b1[i])
        e1.record()
        torch.cuda.synchronize()
        lat1.append(e0.elapsed_time(e1))

    serving = serving32 = None
    if args.serve_requests > 0:
        serving = serve_leg(torch, kfb, dev, args, MIX, args.serve_requests, grouped=True)
        _progress("serving leg (mixed) done")
    if args.serve_requests_fp32 > 0:
        serving32 = serve_leg(torch, kfb, dev, args, kfb.KFB_FP32, args.serve_requests_fp32, grouped=False)
        _progress("serving leg (fp32 plain) done")
    serving_mixed = serve_mixed_leg(torch, kfb, dev, args) if args.serve_requests_uneven > 0 else None
    _progress("uneven serving leg done")

    out = {
        "metric": "B-updates/s + p50/p99 latency, BF16-mixed vs FP32 plain, d=4096 r=256 n=256",
        "value": round(bups, 2),
        "unit": "B-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+fp32+fp64" if refined else "bf16+fp64",
        "data": "synthetic (seeded decaying-spectrum batches and N(0,1) gradients generated on the device)",
        "config": {"workload": f"{L}-layer stack, 2 K-factors per layer ({S} states) at d={D}, r={R}, "
                               f"n={N_BATCH}, rho={RHO}, lambda={LAM}; step = grouped Brand update of all "
                               f"states + grouped two-sided preconditioning of all {L} layers (on two streams: "
                               f"the preconditioning reads the factors of the previous update"
                               + (f"; the update's stream on {cus_upd} CUs, the preconditioning's on {cus_pre})"
                                  if cus_upd else ")"),
                   "layers": L, "states": S, "d": D, "r": R, "n": N_BATCH, "precision": "bf16-mixed",
                   "parallelism": "single-gpu",
                   "streams": ({"update_cus": cus_upd, "precond_cus": cus_pre} if cus_upd else None)},
        "latency_ms": {"step_p50": round(_percentile(step_ms, 50), 3),
                       "step_p99": round(_percentile(step_ms, 99), 3),
                       "single_update_p50": round(_percentile(lat1, 50), 3),
                       "single_update_p99": round(_percentile(lat1, 99), 3),
                       "note": "closed loop; step = 48 updates + 24 preconditionings"},
        "fp32_plain": fp32_plain,
        "fp32_grouped": fp32_grouped,
        "sequential_step": sequential,
        "graph_replay": graph_replay,
        "serving": serving,
        "serving_fp32_plain": serving32,
        "serving_uneven": serving_mixed,
        "roofline": roofline,
        "stages": stages,
        "stages_note": ("per-call stage times inside the timed two-stream step (the preconditioning's "
                        "stages on its CU share); --one-stream gives them in sequence on the whole GPU"),
        "factored_apply": factored,
        "brkfac": brkfac,
        "status_events": sorted(set(status)),
        "autotune": {"jacobi_config": tune.config_name(best_bw) if best_bw else None,
                     "candidates_ms": {tune.config_name(k): round(1e3 * v, 2) for k, v in tune_ms.items()},
                     "precond_gemm_tile": tile_best,
                     "precond_tile_candidates_ms": {str(k): round(1e3 * v, 3) for k, v in tile_ms.items()}},
    }
    out["library"] = kfb.load().kfb_build_info().decode()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        a = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
