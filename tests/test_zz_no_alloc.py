"""mck_fastfood_backward_p_noalloc, the adjoint without device allocation,
against mck_fastfood_backward_p (the same kernels with stream-ordered
temporaries) through the C interface: outputs must be bit-identical, over
two calls in a row on the same static scratch, the second smaller than the
first, plus a dx-only and a parameters-only call.  The allocating call is
itself held to the FP64 oracle by the adjoint parity tests; the first case
here also checks sampled dx rows and the batch sums against the oracle
(1e-5 normwise)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def mk():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_08159_amd as mk

    mk._lib.lib()
    return mk


def _outs(torch, batch, d, n, E, dx=True, params=True):
    nan = float("nan")
    f = lambda *s: torch.full(s, nan, dtype=torch.float32, device="cuda")
    return (f(batch, d) if dx else None,
            f(E, n) if params else None, f(E, n) if params else None, f(E, n) if params else None)


def _case(mk, torch, batch, d, E, seed, sigma, dx=True, params=True, x_np=None):
    n = mk.padded_dim(d)
    p = mk.params(seed, n, E, sigma)
    x_np = workloads.normal(batch, d, seed=batch + d) if x_np is None else x_np
    x = torch.from_numpy(x_np).cuda()
    dphi = torch.from_numpy(workloads.grad_features(batch, 2 * n * E, seed=batch)).cuda()
    ref = mk.backward_p(x, dphi, p["B"], p["perm"], p["G"], p["S"], out=_outs(torch, batch, d, n, E, dx, params))
    got = mk.backward_p(x, dphi, p["B"], p["perm"], p["G"], p["S"], out=_outs(torch, batch, d, n, E, dx, params),
                        noalloc=True)
    torch.cuda.synchronize()
    for name, a, b in zip(("dx", "dB", "dG", "dS"), got, ref):
        if b is None:
            assert a is None
            continue
        assert torch.isfinite(b).all(), name
        assert torch.equal(a, b), (name, float((a - b).abs().max()))
    return x_np, dphi.cpu().numpy(), p, got


def test_noalloc_matches_allocating_call_twice(mk, orc):
    import torch

    # first call: the metric workload (8192 x 784, E = 16, sigma = 2), whose
    # temporaries take most of the static scratch
    batch, d, E, sigma = 8192, 784, 16, 2.0
    print("case: noalloc backward 8192x784 E=16", flush=True)
    x_np = workloads.mnist_sparse(batch)
    x_np, dphi, p, got = _case(mk, torch, batch, d, E, workloads.FASTFOOD_SEED, sigma, x_np=x_np)
    n = 1024
    rows = np.array([0, 31, 4095, 8191])
    P = {k: v.cpu().numpy() for k, v in p.items()}
    rx, rB, rG, rS = orc.backward(x_np[rows].astype(np.float64), dphi[rows].astype(np.float64), n, E, P["B"],
                                  P["perm"], P["G"], P["S64"])
    dx = got[0].cpu().numpy()[rows].astype(np.float64)
    err = np.linalg.norm(dx - rx, axis=1) / np.linalg.norm(rx, axis=1)
    assert err.max() <= TOL, err
    _, rB, rG, rS = orc.backward(x_np.astype(np.float64), dphi, n, E, P["B"], P["perm"], P["G"], P["S64"])
    for name, a, r in (("dB", got[1], rB), ("dG", got[2], rG), ("dS", got[3], rS)):
        e = np.linalg.norm(a.cpu().numpy().astype(np.float64) - r) / np.linalg.norm(r)
        assert e <= TOL, (name, e)
    # second call, smaller: n = 512, split expansions (dx slices in the scratch)
    print("case: noalloc backward 1000x300 E=5", flush=True)
    assert mk.backward_launch_shape(1000, 300, 5)["esplit"] > 1
    _case(mk, torch, 1000, 300, 5, 7, 300 ** 0.5)


def test_noalloc_partial_requests(mk):
    import torch

    print("case: noalloc backward dx only / params only", flush=True)
    _case(mk, torch, 777, 64, 3, 11, 8.0, dx=True, params=False)
    _case(mk, torch, 300, 2000, 2, 12, 40.0, dx=False, params=True)
    _case(mk, torch, 5, 3, 1, 13, 1.0)

