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


def _cu_masked_pair(torch, dev, n_second):
    """Two streams on disjoint CU sets (the benchmark's split), or None if refused."""
    import ctypes
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    hip = ctypes.CDLL("libamdhip64.so")
    words = (ncu + 31) // 32
    out = []
    for cus in (range(0, ncu - n_second), range(ncu - n_second, ncu)):
        mask = (ctypes.c_uint32 * words)()
        for c in cus:
            mask[c // 32] |= 1 << (c % 32)
        h = ctypes.c_void_p()
        if hip.hipExtStreamCreateWithCUMask(ctypes.byref(h), ctypes.c_uint32(words), mask) != 0:
            return None
        out.append(torch.cuda.ExternalStream(h.value, device=dev))
    return out


@pytest.mark.parametrize("masked", [False, True])
def test_two_stream_pipeline_equals_one_stream(kfb, masked):
    # the benchmark's step on two streams: each step's preconditioning (reading the
    # factors the previous update left in the front buffers) runs beside that step's
    # update (writing the back buffers); ordered by events on the buffer they share.
    # Every step's S and every state equal the same calls issued in that order on one
    # stream, bit for bit, with extra work on a third stream to shift the timing; with
    # `masked` the two streams run on disjoint CU sets, as in the benchmark's step.
    import torch
    dev = torch.device("cuda:0")
    d, r, n, L, steps = 768, 96, 64, 3, 5
    prec = kfb.KFB_BF16_MIXED
    print(f"two-stream pipeline: mixed d={d} r={r} n={n} layers={L} steps={steps}", flush=True)

    def group():
        return [kfb.Factor(d, r, n, 0.95, prec) for _ in range(2 * L)]

    A, B = group(), group()
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    k = torch.arange(1, d + 1, device=dev, dtype=torch.float32)
    batches = [[torch.relu(torch.randn(n, d, generator=g, device=dev) * k ** -1.0).to(torch.bfloat16)
                for _ in range(2 * L)] for _ in range(steps + 1)]
    Gs = [[torch.randn(d, d, generator=g, device=dev) for _ in range(L)] for _ in range(steps)]
    SA = [[torch.empty(d, d, device=dev) for _ in range(L)] for _ in range(steps)]
    SB = [[torch.empty(d, d, device=dev) for _ in range(L)] for _ in range(steps)]
    wsA, wsB, wsP = kfb.Workspace(), kfb.Workspace(), kfb.Workspace()
    lam = [0.01] * L
    for grp, ws in ((A, wsA), (B, wsB)):
        kfb.update_batched(grp, batches[0], ws)
    torch.cuda.synchronize()
    # reference: one stream, preconditioning then update at every step
    for j in range(steps):
        kfb.precondition_batched(A[1::2], A[0::2], Gs[j], SA[j], lam, lam, 0, wsA)
        kfb.update_batched(A, batches[j + 1], wsA)
    # pipeline: two streams (unmasked, or on disjoint CU sets as in the benchmark),
    # plus unrelated work on a third
    s_upd, s_pre = torch.cuda.current_stream(), torch.cuda.Stream(device=dev)
    if masked:
        pair = _cu_masked_pair(torch, dev, 64)
        assert pair is not None, "the runtime refused the CU-masked streams"
        s_upd, s_pre = pair
    s_noise = torch.cuda.Stream(device=dev)
    big = torch.randn(2048, 2048, device=dev)
    eu = ep = None
    for j in range(steps):
        with torch.cuda.stream(s_noise):
            for _ in range(4):
                big = big @ big
                big = big / big.norm()
        with torch.cuda.stream(s_pre):
            if eu is not None:
                s_pre.wait_event(eu)
            kfb.precondition_batched(B[1::2], B[0::2], Gs[j], SB[j], lam, lam, 0, wsP)
            ep = torch.cuda.Event()
            ep.record(s_pre)
        with torch.cuda.stream(s_upd):
            if j > 0:
                s_upd.wait_event(prev_ep)
            kfb.update_batched(B, batches[j + 1], wsB)
            eu = torch.cuda.Event()
            eu.record(s_upd)
        prev_ep = ep
    s_upd.wait_stream(s_pre)
    torch.cuda.synchronize()
    if masked:  # each masked stream holds a hardware queue: give them back
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        for st in (s_upd, s_pre):
            hip.hipStreamDestroy(ctypes.c_void_p(st.cuda_stream))
    print(f"  two-stream pipeline (masked={masked}) done", flush=True)
    for j in range(steps):
        for x, y in zip(SA[j], SB[j]):
            assert torch.equal(x, y), f"step {j}: preconditioned gradient differs"
    for fa, fb in zip(A, B):
        Ua, Da = fa.front()
        Ub, Db = fb.front()
        assert torch.equal(Ua, Ub) and torch.equal(Da, Db)
    assert all(f.status() == 0 for f in A + B)
