"""The library's temporaries (backward partial sums and dx slices, the
training step's scratch) come from cached blocks shared by every call on a
device.  These tests check, through the C ABI, that

* calls alternating between two streams, whose blocks therefore move from
  one stream to the other behind a device-side event wait, give exactly the
  results of the same calls made alone (the adjoint's sums have a fixed
  order, so the comparison is bit for bit);
* a call returns to the host while earlier work is still queued on its
  stream: taking a temporary never waits on the host.
"""
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_08159_amd as mk

    mk._lib.lib()
    return mk, torch


def _inputs(torch, seed, batch, d, n, E):
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.standard_normal((batch, d)).astype(np.float32)).cuda()
    g = torch.from_numpy(rng.standard_normal((batch, 2 * n * E)).astype(np.float32)).cuda()
    return x, g


@pytest.mark.parametrize("batch,d,E", [(1024, 784, 16), (300, 100, 3), (5000, 784, 4)])
def test_backward_on_two_streams_matches_single_calls(env, batch, d, E):
    mk, torch = env
    n = mk.padded_dim(d)
    a = _inputs(torch, 11, batch, d, n, E)
    b = _inputs(torch, 12, batch, d, n, E)
    print("backward on two streams: batch %d d %d E %d" % (batch, d, E), flush=True)
    ref_a = mk.backward(a[0], a[1], E, seed=5, sigma=2.0, need_params=True)
    ref_b = mk.backward(b[0], b[1], E, seed=5, sigma=2.0, need_params=True)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for k in range(6):
        s, (x, g) = (sa, a) if k % 2 == 0 else (sb, b)
        with torch.cuda.stream(s):
            outs.append(mk.backward(x, g, E, seed=5, sigma=2.0, need_params=True))
    torch.cuda.synchronize()
    for k, got in enumerate(outs):
        ref = ref_a if k % 2 == 0 else ref_b
        for r, o in zip(ref, got):
            assert torch.equal(r, o), k


@pytest.mark.parametrize("d,batch,E", [(131067, 3, 2), (262144, 2, 1)])
def test_long_forward_on_two_streams_matches_single_calls(env, d, batch, E):
    # the long-vector path's scratch rows are temporaries too
    mk, torch = env
    rng = np.random.default_rng(21)
    xa = torch.from_numpy(rng.standard_normal((batch, d)).astype(np.float32)).cuda()
    xb = torch.from_numpy(rng.standard_normal((batch + 1, d)).astype(np.float32)).cuda()
    print("long forward on two streams: d %d batch %d E %d" % (d, batch, E), flush=True)
    ref_a = mk.forward(xa, E, 9, 1.5)
    ref_b = mk.forward(xb, E, 9, 1.5)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for k in range(4):
        s, x = (sa, xa) if k % 2 == 0 else (sb, xb)
        with torch.cuda.stream(s):
            outs.append(mk.forward(x, E, 9, 1.5))
    torch.cuda.synchronize()
    for k, got in enumerate(outs):
        assert torch.equal(got, ref_a if k % 2 == 0 else ref_b), k


def _host_ms_behind_busy_stream(torch, call, busy_cycles=200_000_000):
    torch.cuda.synchronize()
    torch.cuda._sleep(busy_cycles)  # tens of milliseconds of queued work
    t0 = time.perf_counter()
    call()
    host_ms = (time.perf_counter() - t0) * 1e3
    s0 = time.perf_counter()
    torch.cuda.synchronize()
    drain_ms = (time.perf_counter() - s0) * 1e3
    return host_ms, drain_ms


def test_calls_with_temporaries_do_not_wait_on_the_host(env):
    mk, torch = env
    batch, d, n, E, C = 1024, 784, 1024, 16, 10
    x, g = _inputs(torch, 13, batch, d, n, E)
    p = mk.params(workloads.FASTFOOD_SEED, n, E, 1.0)
    B, perm, G, S = (t.contiguous() for t in (p["B"], p["perm"], p["G"], p["S"]))
    W = torch.zeros((C, 2 * n * E), device="cuda")
    bias = torch.zeros(C, device="cuda")
    labels = torch.from_numpy(np.arange(batch, dtype=np.int32) % C).cuda()
    calls = {
        "backward": lambda: mk.backward(x, g, E, seed=5, sigma=2.0, need_params=True),
        "train_step": lambda: mk.train_step(x, labels, W, bias, B, perm, G, S),
    }
    for name, call in calls.items():
        call()
        call()  # the temporaries exist now
        host_ms, drain_ms = _host_ms_behind_busy_stream(torch, call)
        print("%s: host %.2f ms, stream drained %.2f ms later" % (name, host_ms, drain_ms), flush=True)
        # the queued work takes tens of milliseconds: a call that waited for
        # it would return only after it, leaving nothing to drain
        assert drain_ms > 10.0 and host_ms < drain_ms, (name, host_ms, drain_ms)


def test_calls_with_temporaries_replay_from_a_graph(env):
    # under capture the temporaries are graph-owned allocations: every
    # replay, with eager calls (which use the cached blocks) and
    # synchronisation in between, reproduces the eager results bit for bit
    mk, torch = env
    batch, d, n, E, C = 1024, 784, 1024, 16, 10
    x, g = _inputs(torch, 14, batch, d, n, E)
    p = mk.params(workloads.FASTFOOD_SEED, n, E, 1.0)
    B, perm, G, S = (t.contiguous() for t in (p["B"], p["perm"], p["G"], p["S"]))
    W = torch.from_numpy(np.random.default_rng(15).standard_normal((C, 2 * n * E)).astype(np.float32) * 0.01).cuda()
    bias = torch.zeros(C, device="cuda")
    labels = torch.from_numpy(np.arange(batch, dtype=np.int32) % C).cuda()
    ref_b = [t.clone() for t in mk.backward(x, g, E, seed=5, sigma=2.0, need_params=True)]
    ref_t = {k: v.clone() for k, v in mk.train_step(x, labels, W, bias, B, perm, G, S).items() if v is not None}
    torch.cuda.synchronize()
    outb = tuple(torch.empty_like(t) for t in ref_b)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mk.backward(x, g, E, seed=5, sigma=2.0, out=outb)
        mk.train_step(x, labels, W, bias, B, perm, G, S)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    print("capturing backward and training step", flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        mk.backward(x, g, E, seed=5, sigma=2.0, out=outb)
        outt = mk.train_step(x, labels, W, bias, B, perm, G, S)
    for k in range(3):
        for t in outb:
            t.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        for r, o in zip(ref_b, outb):
            assert torch.equal(r, o), ("backward", k)
        for name, r in ref_t.items():
            assert torch.equal(r, outt[name]), (name, k)
        mk.backward(x[:100], g[:100], E, seed=5, sigma=2.0, need_params=True)  # eager work between replays
        torch.cuda.synchronize()
