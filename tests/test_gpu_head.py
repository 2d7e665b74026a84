"""GPU parity of the classifier head's two products (section "Empirical
Analysis and Experiments": softmax(W phi + b) on the McKernel features)
against FP64 numpy.

Each result is a sum of F (or batch) FP32 products; the kernels sum in a
fixed order (per-thread runs, then a tree), so every entry is held to
1e-5 times the sum of the absolute values of its terms, well above the
run-length times the unit roundoff of those orders, and must repeat bit
for bit."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SHAPES = [(1, 4, 1), (3, 8, 10), (37, 4100, 10), (5, 1000, 16), (300, 2052, 7), (1024, 32768, 10)]


@pytest.fixture(scope="module")
def mk():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_08159_amd as mk

    mk._lib.lib()
    return mk


def _inputs(batch, F, C):
    phi = workloads.normal(batch, F, seed=F) * np.float32(0.05)
    W = workloads.normal(C, F, seed=F + 1) * np.float32(0.01)
    b = workloads.normal(1, C, seed=F + 2)[0]
    dl = workloads.normal(batch, C, seed=F + 3) * np.float32(1e-3)
    return phi, W, b, dl


def _close(got, ref, bound):
    got = np.asarray(got, np.float64)
    assert got.shape == ref.shape
    assert np.all(np.abs(got - ref) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("batch,F,C", SHAPES)
def test_head_logits(mk, batch, F, C):
    import torch

    phi, W, b, _ = _inputs(batch, F, C)
    tp, tW, tb = (torch.from_numpy(a).cuda() for a in (phi, W, b))
    got = mk.head_logits(tp, tW, tb).cpu().numpy()
    p64, W64 = phi.astype(np.float64), W.astype(np.float64)
    ref = p64 @ W64.T + b.astype(np.float64)
    bound = np.abs(p64) @ np.abs(W64).T + np.abs(b.astype(np.float64))
    _close(got, ref, bound)
    assert np.array_equal(mk.head_logits(tp, tW, tb).cpu().numpy(), got)
    nob = mk.head_logits(tp, tW).cpu().numpy()
    _close(nob, p64 @ W64.T, np.abs(p64) @ np.abs(W64).T)


@pytest.mark.parametrize("batch,F,C", SHAPES)
def test_head_backward(mk, batch, F, C):
    import torch

    phi, W, _, dl = _inputs(batch, F, C)
    tp, tW, tdl = (torch.from_numpy(a).cuda() for a in (phi, W, dl))
    dphi, dW = mk.head_backward(tp, tdl, tW)
    p64, W64, d64 = phi.astype(np.float64), W.astype(np.float64), dl.astype(np.float64)
    _close(dphi.cpu().numpy(), d64 @ W64, np.abs(d64) @ np.abs(W64))
    _close(dW.cpu().numpy(), d64.T @ p64, np.abs(d64).T @ np.abs(p64))
    dphi2, dW2 = mk.head_backward(tp, tdl, tW)
    assert torch.equal(dphi, dphi2) and torch.equal(dW, dW2)
    # each output alone is the same as both together
    only_dphi, none = mk.head_backward(tp, tdl, tW, need_dW=False)
    assert none is None and torch.equal(only_dphi, dphi)
    none, only_dW = mk.head_backward(tp, tdl, tW, need_dphi=False)
    assert none is None and torch.equal(only_dW, dW)


def test_head_empty_batch_and_refusals(mk):
    import torch

    W = torch.ones((10, 16), device="cuda")
    phi = torch.zeros((0, 16), device="cuda")
    dl = torch.zeros((0, 10), device="cuda")
    dphi, dW = mk.head_backward(phi, dl, W)
    assert dphi.shape == (0, 16) and torch.equal(dW, torch.zeros_like(W))
    assert mk.head_logits(phi, W).shape == (0, 10)
    # 17 classes, unaligned phi, F not a multiple of 4
    with pytest.raises(mk.MckError):
        mk.head_logits(torch.zeros((2, 16), device="cuda"), torch.zeros((17, 16), device="cuda"))
    buf = torch.zeros(2 * 16 + 1, device="cuda")
    with pytest.raises(mk.MckError):
        mk.head_logits(buf[1:].view(2, 16), W)
    with pytest.raises(mk.MckError):
        mk.head_logits(torch.zeros((2, 18), device="cuda"), torch.zeros((10, 18), device="cuda"))
