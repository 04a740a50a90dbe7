"""Continuous-batching request loop: every result equals the same request run
alone (bit for bit: grouped launches are deterministic and shape-keyed),
per-state order holds, a tiny byte budget still drains, and an over-budget
request fails cleanly while the rest are served."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _layers():
    # uneven widths and ranks (r + n_max <= d for every factor)
    return [(256, 384, 64, 32), (384, 512, 32, 64), (512, 256, 64, 64), (256, 256, 32, 32)]


def _make_inputs(torch, dev, layers, n, seed):
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    ins = {}
    for l, (d_in, d_out, _, _) in enumerate(layers):
        for side, d in (("A", d_in), ("G", d_out)):
            k = torch.arange(1, d + 1, device=dev, dtype=torch.float32)
            ins[(l, side)] = [(torch.randn(n, d, generator=g, device=dev) * k ** -0.8).to(torch.bfloat16)
                              for _ in range(3)]
        ins[(l, "grad")] = torch.randn(d_out, d_in, generator=g, device=dev)
    return ins


def _snap(f, stream):
    import torch
    with torch.cuda.stream(stream):
        U, D = f.front()
        return U.clone(), D.clone(), f.info()["k_valid"], f.info()["step"]


def test_alone_equals_mix(kfb):
    import torch
    from paper_2210_08494_amd import serve
    dev = torch.device("cuda:0")
    layers = _layers()
    n = 32
    srv = serve.Server(layers, n_max=n, rho=0.95, prec=kfb.KFB_BF16_MIXED, streams=3)
    ins = _make_inputs(torch, dev, layers, n, seed=5)
    torch.cuda.synchronize()
    # warm every state to r + n modes
    for l in range(len(layers)):
        for side in ("A", "G"):
            for j in range(2):
                srv.submit(serve.UpdateRequest(l, side, ins[(l, side)][j]))
    srv.drain()
    torch.cuda.synchronize()
    pre, post = {}, {}

    def before(kind, reqs, stream):
        for r in reqs:
            pre[r.rid] = [_snap(f, stream) for f in srv._states_of(r)]

    def after(kind, reqs, stream):
        for r in reqs:
            if kind == "U":
                post[r.rid] = _snap(srv._states_of(r)[0], stream)
            else:
                with torch.cuda.stream(stream):
                    post[r.rid] = r.S.clone()

    srv.hooks_before_issue, srv.hooks_after_issue = before, after
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(60):
        l = int(rng.integers(len(layers)))
        if rng.random() < 0.7:
            side = "A" if rng.random() < 0.5 else "G"
            r = serve.UpdateRequest(l, side, ins[(l, side)][int(rng.integers(3))])
        else:
            S = torch.empty_like(ins[(l, "grad")])
            r = serve.PrecondRequest(l, ins[(l, "grad")], S, 0.01, 0.02)
        reqs.append(r)
        srv.submit(r)
        if i % 7 == 6:
            srv.step()
    srv.drain()
    torch.cuda.synchronize()
    assert srv.stats.completed >= 60 and srv.stats.groups < srv.stats.completed  # some grouping happened
    ws = kfb.Workspace(dev)
    checked = 0
    for r in reqs:
        states = [(f.d, f.r, f.n_max) for f in srv._states_of(r)]
        alone = []
        for (d, rr, nm), (U, D, k, step) in zip(states, pre[r.rid]):
            f = kfb.Factor(d, rr, nm, 0.95, kfb.KFB_BF16_MIXED, device=dev)
            f.load_state(U, D, step=step)
            alone.append(f)
        if isinstance(r, serve.UpdateRequest):
            alone[0].update(r.M, ws)
            torch.cuda.synchronize()
            Ua, Da = alone[0].front()
            Um, Dm, km, sm = post[r.rid]
            assert torch.equal(Ua, Um) and torch.equal(Da, Dm), f"update {r.rid} differs alone vs mix"
        else:
            S = torch.empty_like(r.S)
            kfb.precondition(alone[0], alone[1], r.G, S, r.lam_g, r.lam_a, ws=ws)
            torch.cuda.synchronize()
            assert torch.equal(S, post[r.rid]), f"precondition {r.rid} differs alone vs mix"
        checked += 1
    assert checked == 60


def test_tiny_budget_and_rejection(kfb):
    import torch
    from paper_2210_08494_amd import serve
    dev = torch.device("cuda:0")
    layers = _layers()[:2] + [(2048, 2048, 32, 32)]
    n = 32
    ins = _make_inputs(torch, dev, layers, n, seed=9)
    srv = serve.Server(layers, n_max=n, prec=kfb.KFB_BF16_MIXED)
    torch.cuda.synchronize()
    for j in range(2):  # warm every state to its steady shape
        for l in range(3):
            for side in ("A", "G"):
                srv.submit(serve.UpdateRequest(l, side, ins[(l, side)][j]))
    srv.drain()
    torch.cuda.synchronize()
    # budget: the largest single steady-state update of the two small layers
    budget = max(srv._bytes_for(srv._key(r), [r])
                 for r in (serve.UpdateRequest(l, s, ins[(l, s)][0]) for l in range(2) for s in ("A", "G")))
    bad = serve.PrecondRequest(2, ins[(2, "grad")], torch.empty_like(ins[(2, "grad")]))
    assert srv._bytes_for(srv._key(bad), [bad]) > budget
    srv.byte_budget = budget
    srv.stats = serve.ServerStats()
    order = []
    for rep in range(3):
        for l in range(2):
            for side in ("A", "G"):
                r = serve.UpdateRequest(l, side, ins[(l, side)][rep])
                order.append(r)
                srv.submit(r)
        if rep == 1:
            srv.submit(bad)
    srv.drain()
    torch.cuda.synchronize()
    assert srv.stats.max_inflight_bytes <= budget
    assert srv.stats.completed == len(order)
    assert bad.error and srv.stats.rejected == 1
    # per-state order kept and nothing lost: each small state saw 2 + 3 updates
    for l in range(2):
        for side in ("A", "G"):
            assert srv.factor(l, side).info()["step"] == 5


# ----------------------------------------------------------------------------
# The serving mix at the shapes of the batched-serving workload: widths from
# {512, ..., 8192}, ranks from {64, ..., 512} (clamped to d - n_max), batch
# widths from {64, 128, 256}, padded groups of uneven widths, preconditionings
# with and without spectrum continuation.  Every served result is checked
# against the FP64 oracle replaying the same per-state sequence, and against
# the same request run alone from the state it found.
# ----------------------------------------------------------------------------
def _c4_layers():
    widths = [1024, 2048, 512, 4096, 1024]
    ranks = [256, 128, 512, 64]
    nmax = 256
    return [(widths[l], widths[l + 1], min(ranks[l], widths[l] - nmax), min(ranks[l], widths[l + 1] - nmax))
            for l in range(4)], nmax


@pytest.mark.timeout(600)
def test_config4_shapes_padded_groups_vs_oracle_and_alone(kfb):
    import torch
    import oracle
    from paper_2210_08494_amd import serve, synth
    dev = torch.device("cuda:0")
    layers, nmax = _c4_layers()
    rho, lam = 0.95, 0.01
    srv = serve.Server(layers, n_max=nmax, rho=rho, prec=kfb.KFB_BF16_MIXED, streams=3, pad_updates=True)
    orc = {}
    for l, (d_in, d_out, r_a, r_g) in enumerate(layers):
        orc[(l, "A")] = oracle.BrandFactor(d_in, r_a, rho)
        orc[(l, "G")] = oracle.BrandFactor(d_out, r_g, rho)

    def batch(tag, l, side, n):
        d = layers[l][0] if side == "A" else layers[l][1]
        x = synth.to_bf16_values(synth.batch_for(700 + tag, l, side, n, d))
        return x, torch.from_numpy(x).to(device=dev, dtype=torch.bfloat16)

    seq = []   # (request, host batch) in submission order: the oracle replays it
    for j in range(2):
        for l in range(len(layers)):
            for side in ("A", "G"):
                x, xd = batch(j, l, side, nmax)
                r = serve.UpdateRequest(l, side, xd)
                seq.append((r, x))
                srv.submit(r)
    srv.drain()
    torch.cuda.synchronize()
    pre, post = {}, {}

    def before(kind, reqs, stream):
        for r in reqs:
            pre[r.rid] = [_snap(f, stream) for f in srv._states_of(r)]

    def after(kind, reqs, stream):
        for r in reqs:
            if kind == "U":
                post[r.rid] = _snap(srv._states_of(r)[0], stream)
            else:
                with torch.cuda.stream(stream):
                    post[r.rid] = r.S.clone()

    srv.hooks_before_issue, srv.hooks_after_issue = before, after
    rng = np.random.default_rng(44)
    grads = {}
    for i in range(48):
        l = int(rng.integers(len(layers)))
        if rng.random() < 0.65:
            side = "A" if rng.random() < 0.5 else "G"
            n = int(rng.choice([64, 128, 256]))
            x, xd = batch(10 + i, l, side, n)
            r = serve.UpdateRequest(l, side, xd)
            seq.append((r, x))
        else:
            if l not in grads:
                d_in, d_out = layers[l][:2]
                grads[l] = torch.from_numpy(synth.grad_for(745, l, d_out, d_in).astype(np.float32)).to(dev)
            flags = int(rng.integers(2))   # with and without spectrum continuation
            r = serve.PrecondRequest(l, grads[l], torch.empty_like(grads[l]), lam, lam, flags)
            seq.append((r, None))
        srv.submit(r)
        if i % 5 == 4:
            srv.step()
    srv.drain()
    torch.cuda.synchronize()
    assert srv.stats.grouped_problems > srv.stats.groups     # some requests shared a launch sequence
    ws = kfb.Workspace(dev)
    worst = dict(alone=0.0, rec=0.0, S=0.0, S_proj=0.0, S_alone=0.0)
    for r, x in seq:
        if isinstance(r, serve.UpdateRequest):
            o = orc[(r.layer, r.side)]
            o.update(x.T)
            if r.rid not in post:
                continue        # warm-up: no snapshot
            f = srv.factor(r.layer, r.side)
            (U0, D0, k0, s0), = pre[r.rid]
            alone = kfb.Factor(f.d, f.r, f.n_max, rho, kfb.KFB_BF16_MIXED, device=dev)
            alone.load_state(U0, D0, step=s0)
            alone.update(r.M, ws)
            torch.cuda.synchronize()
            Ua, Da = alone.front()
            Um, Dm, km, sm = post[r.rid]
            Ua, Da, Um, Dm = (t.double().cpu().numpy() for t in (Ua, Da, Um, Dm))
            worst["alone"] = max(worst["alone"], oracle.e_rec_lowrank(Um, Dm, Ua, Da))
            worst["rec"] = max(worst["rec"], oracle.e_rec_lowrank(Um, Dm, o.U, o.D))
        else:
            og, oa = orc[(r.layer, "G")], orc[(r.layer, "A")]
            DG, lg = (oracle.spectrum_continuation(og.D, lam) if r.flags else (og.D, lam))
            DA, la = (oracle.spectrum_continuation(oa.D, lam) if r.flags else (oa.D, lam))
            G = r.G.double().cpu().numpy()
            ref = oracle.precondition_lowrank(og.U, DG, oa.U, DA, G, lg, la)
            Sm = post[r.rid].double().cpu().numpy()
            worst["S"] = max(worst["S"], oracle.e_S(Sm, ref))
            worst["S_proj"] = max(worst["S_proj"], oracle.e_S_proj(Sm, ref, og.U, oa.U))
            fs = []
            for f, (U0, D0, k0, s0) in zip(srv._states_of(r), pre[r.rid]):
                a = kfb.Factor(f.d, f.r, f.n_max, rho, kfb.KFB_BF16_MIXED, device=dev)
                a.load_state(U0, D0, step=s0)
                fs.append(a)
            S = torch.empty_like(r.S)
            kfb.precondition(fs[0], fs[1], r.G, S, lam, lam, r.flags, ws=ws)
            torch.cuda.synchronize()
            worst["S_alone"] = max(worst["S_alone"], oracle.e_S(Sm, S.double().cpu().numpy()))
    print(f"  config-4 serving mix: {worst}", flush=True)
    assert worst["rec"] <= 2e-2 and worst["S"] <= 2e-2 and worst["S_proj"] <= 2e-2
    assert worst["alone"] <= 1e-4 and worst["S_alone"] <= 1e-4


def test_inputs_produced_on_the_submitters_stream(kfb):
    # a backward pass writes M (and G) on its own stream and submits at once: the
    # group must wait for that work (the server records an event at submit)
    import torch
    from paper_2210_08494_amd import serve
    dev = torch.device("cuda:0")
    layers = [(512, 512, 64, 64)]
    n = 64
    ins = _make_inputs(torch, dev, layers, n, seed=21)
    srv = serve.Server(layers, n_max=n, prec=kfb.KFB_BF16_MIXED, streams=2)
    twin = kfb.Factor(512, 64, n, 0.95, kfb.KFB_BF16_MIXED, device=dev)
    for j in range(2):
        srv.submit(serve.UpdateRequest(0, "A", ins[(0, "A")][j]))
        srv.submit(serve.UpdateRequest(0, "G", ins[(0, "G")][j]))
        twin.update(ins[(0, "A")][j])
    srv.drain()
    torch.cuda.synchronize()
    producer = torch.cuda.Stream(device=dev)
    M = torch.zeros_like(ins[(0, "A")][2])
    S = torch.empty_like(ins[(0, "grad")])
    Gbuf = torch.zeros_like(ins[(0, "grad")])
    big = torch.randn(4096, 4096, device=dev)
    with torch.cuda.stream(producer):
        for _ in range(30):                 # keep the producer busy before it writes the inputs
            big = big @ big
            big = big / big.norm()
        M.copy_(ins[(0, "A")][2])
        Gbuf.copy_(ins[(0, "grad")])
        srv.submit(serve.UpdateRequest(0, "A", M))
        srv.submit(serve.PrecondRequest(0, Gbuf, S, 0.01, 0.02))
    srv.drain()
    torch.cuda.synchronize()
    twin.update(ins[(0, "A")][2])
    Ua, Da = srv.factor(0, "A").front()
    Ub, Db = twin.front()
    assert torch.equal(Ua, Ub) and torch.equal(Da, Db)
    S2 = torch.empty_like(S)
    kfb.precondition(srv.fg[0], srv.fa[0], ins[(0, "grad")], S2, 0.01, 0.02)
    torch.cuda.synchronize()
    assert torch.equal(S, S2)
