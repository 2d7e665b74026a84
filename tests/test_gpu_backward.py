"""GPU parity of the adjoint (dx and the batch sums dB, dG, dS) against the
FP64 oracle in every launch shape the library uses: one or several row
passes per block, expansions split over block groups, and the full metric
workload (8192 x 784, E = 16, sigma = 2) in exactly the shape the benchmark
times.  The shape of each case is read from the library
(mck_backward_launch_shape) and asserted, so a change of geometry cannot
silently move a case off the path it is meant to cover.

Tolerance: 1e-5 normwise, per row for dx and per tensor for dB, dG, dS (the
FP32 target of the method).  dx is compared on sampled rows, always
including the first and last row of every pass of the first, a middle and
the last block; dB, dG, dS are compared over the whole batch.
"""
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


def rowwise_rel(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref, axis=1)
    den[den == 0] = 1.0
    return np.linalg.norm(a - ref, axis=1) / den


def tensor_rel(a, ref):
    return float(np.linalg.norm(np.asarray(a, np.float64) - ref) / max(np.linalg.norm(ref), 1e-300))


def boundary_rows(shape, batch, extra=16, seed=0):
    """First and last row of every pass of the first, a middle and the last
    row block, plus `extra` random rows."""
    R, P, NB = shape["rows_per_pass"], shape["passes"], shape["rowblocks"]
    rows = set()
    for b in sorted({0, NB // 2, NB - 1}):
        for p in range(P):
            r0 = (b * P + p) * R
            for r in (r0, r0 + R - 1):
                if r < batch:
                    rows.add(r)
    rows.update(np.random.default_rng(seed).choice(batch, size=min(extra, batch), replace=False).tolist())
    rows.add(batch - 1)
    return np.array(sorted(rows))


def run_case(mk, orc, x, dphi, E, seed, sigma, shape, full_params=True):
    import torch

    batch, d = x.shape
    n = mk.padded_dim(d)
    dx, dB, dG, dS = mk.backward(torch.from_numpy(x).cuda(), torch.from_numpy(dphi).cuda(), E, seed, sigma,
                                 need_dx=True, need_params=True)
    torch.cuda.synchronize()
    p = orc.params(seed, n, E, sigma)
    rows = boundary_rows(shape, batch)
    rx = orc.backward(x[rows].astype(np.float64), dphi[rows].astype(np.float64), n, E, p["B"], p["perm"],
                      p["G"], p["S64"])[0]
    err_dx = rowwise_rel(dx.cpu().numpy()[rows], rx)
    assert err_dx.max() <= TOL, (rows[np.argmax(err_dx)], err_dx.max())
    if full_params:
        _, rB, rG, rS = orc.backward(x.astype(np.float64), dphi, n, E, p["B"], p["perm"], p["G"], p["S64"])
        for name, got, ref in (("dB", dB, rB), ("dG", dG, rG), ("dS", dS, rS)):
            e = tensor_rel(got.cpu().numpy(), ref)
            assert e <= TOL, (name, e)
    return dx


def test_backward_metric_workload_bench_shape(mk, orc):
    # the adjoint of the benchmark's fwd+bwd figure: 8192 x 784, E = 16,
    # sigma = 2, the paper's seed; four row passes per block, 256 blocks
    batch, d, E, sigma = 8192, 784, 16, 2.0
    shape = mk.backward_launch_shape(batch, d, E)
    assert shape == {"rows_per_pass": 8, "passes": 4, "esplit": 1, "rowblocks": 256}, shape
    x = workloads.mnist_sparse(batch)
    dphi = workloads.grad_features(batch, 2 * 1024 * E)
    print("case: metric backward 8192x784 E=16 shape %s" % shape, flush=True)
    run_case(mk, orc, x, dphi, E, workloads.FASTFOOD_SEED, sigma, shape)


# (d, batch, E, expected passes, expected esplit): batches just past each
# passes threshold at n = 64, 256, 1024, with and without split expansions
SWEEP = [
    (784, 2049, 3, 2, 2),     # n = 1024: 257 row units -> 2 passes, 129 blocks, 2 expansion groups
    (784, 4097, 2, 3, 2),     # 3 passes, 171 blocks
    (784, 6145, 2, 4, 2),     # 4 passes, 193 blocks
    (784, 8200, 1, 4, 1),     # past the LDS limit of 4 passes: 257 blocks
    (1024, 8193, 1, 3, 1),    # d = n: the dx rows take more LDS, 3 passes at most
    (256, 8193, 2, 2, 2),     # n = 256: 32 rows per pass
    (200, 16385, 3, 3, 2),    # n = 256, ragged d
    (64, 32769, 2, 2, 2),     # n = 64: 128 rows per pass
    (33, 65537, 1, 3, 1),     # n = 64, ragged d, 3 passes
]


@pytest.mark.parametrize("d,batch,E,passes,esplit", SWEEP)
def test_backward_passes_sweep(mk, orc, d, batch, E, passes, esplit):
    shape = mk.backward_launch_shape(batch, d, E)
    assert (shape["passes"], shape["esplit"]) == (passes, esplit), shape
    n = mk.padded_dim(d)
    x = workloads.normal(batch, d, seed=d + batch)
    dphi = workloads.grad_features(batch, 2 * n * E, seed=batch)
    print("case: backward d=%d batch=%d E=%d shape %s" % (d, batch, E, shape), flush=True)
    run_case(mk, orc, x, dphi, E, 91, float(n) ** 0.5, shape)


def test_backward_empty_batch_zeroes_parameter_gradients(mk):
    # the sums over an empty batch are zero; every entry point writes them
    # (with a fill kernel, so the call can be captured into a graph)
    import torch

    E, d = 3, 100
    n = mk.padded_dim(d)
    x = torch.zeros((0, d), device="cuda")
    g = torch.zeros((0, 2 * n * E), device="cuda")
    p = mk.params(3, n, E, 1.0)
    B, perm, G, S = (p[k].contiguous() for k in ("B", "perm", "G", "S"))
    calls = {
        "seed": lambda out: mk.backward(x, g, E, seed=3, sigma=1.0, out=out),
        "explicit": lambda out: mk.backward_p(x, g, B, perm, G, S, out=out),
        "explicit without allocation": lambda out: mk.backward_p(x, g, B, perm, G, S, out=out, noalloc=True),
    }
    for name, call in calls.items():
        print("empty batch:", name, flush=True)
        out = (torch.empty((0, d), device="cuda"),) + tuple(
            torch.full((E, n), float("nan"), device="cuda") for _ in range(3))
        call(out)
        torch.cuda.synchronize()
        for o in out[1:]:
            assert bool((o == 0).all()), name
