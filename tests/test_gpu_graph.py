"""Grouped calls captured into a HIP graph (torch.cuda.CUDAGraph) do the same
work as the eager calls.

The library only launches kernels on the caller's stream (the per-problem
record table goes up through a kernel whose arguments carry it), so a group's
calls can be captured.  A Brand update writes the state's back buffer and
then makes it the front, so the captured sequence holds two consecutive
updates (the buffers trade roles twice and end as they started) and a grouped
preconditioning; it is replayed several times with eager work and
synchronisation in between, and every replay must equal the same eager
sequence on a twin group bit for bit.
"""
import pytest

pytestmark = pytest.mark.gpu


def test_graph_replay_equals_eager(kfb):
    import torch
    dev = torch.device("cuda:0")
    d, r, n, L = 512, 64, 64, 3
    prec = kfb.KFB_BF16_MIXED
    print(f"graph replay: mixed d={d} r={r} n={n} layers={L}", flush=True)

    def group():
        return [kfb.Factor(d, r, n, 0.95, prec) for _ in range(2 * L)]

    A, B = group(), group()
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    k = torch.arange(1, d + 1, device=dev, dtype=torch.float32)
    batches = [[torch.relu(torch.randn(n, d, generator=g, device=dev) * k ** -1.0).to(torch.bfloat16)
                for _ in range(2 * L)] for _ in range(2)]
    Gs = [torch.randn(d, d, generator=g, device=dev) for _ in range(L)]
    SA = [torch.empty(d, d, device=dev) for _ in range(L)]
    SB = [torch.empty(d, d, device=dev) for _ in range(L)]
    wsA, wsB = kfb.Workspace(), kfb.Workspace()

    def seq(states, ws, S):
        kfb.update_batched(states, batches[0], ws)
        kfb.update_batched(states, batches[1], ws)
        kfb.precondition_batched(states[1::2], states[0::2], Gs, S, [0.01] * L, [0.01] * L, 0, ws)

    # warm-up on both twins: r + n modes reached, workspaces sized, kernel attributes set
    seq(A, wsA, SA)
    seq(B, wsB, SB)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        seq(B, wsB, SB)
    torch.cuda.synchronize()
    for rep in range(3):
        seq(A, wsA, SA)
        graph.replay()
        torch.cuda.synchronize()
        for fa, fb in zip(A, B):
            Ua, Da = fa.front()
            Ub, Db = fb.front()
            assert torch.equal(Ua, Ub) and torch.equal(Da, Db), f"replay {rep}: state differs"
        for x, y in zip(SA, SB):
            assert torch.equal(x, y), f"replay {rep}: preconditioned gradient differs"
        print(f"  replay {rep} equal", flush=True)
    assert all(f.status() == 0 for f in A + B)
