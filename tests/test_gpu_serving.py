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
