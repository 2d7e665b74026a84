"""GPU parity of the RBF-Matern calibration (section "Customizing McKernel")
against the FP64 oracle: the generated S (FP64 and FP32) bit for bit, and
the feature map built on it within the FP32 tolerance (1e-5 per row)."""
import functools
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SEED = workloads.FASTFOOD_SEED


@pytest.fixture(scope="module")
def mk():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_08159_amd as mk

    mk._lib.lib()
    return mk


@functools.lru_cache(maxsize=None)
def _oracle_params(n, E, sigma, t):
    import oracle

    oracle.build(force=False)
    return oracle.params(SEED, n, E, sigma, matern_t=t)


@pytest.mark.parametrize("n,E,sigma,t", [(2, 3, 1.0, 40), (16, 3, 1.0, 40), (64, 2, 0.5, 40), (256, 2, 1.0, 7),
                                         (1024, 1, 1.0, 40), (2048, 1, 2.0, 1)])
def test_matern_params_bit_exact(mk, n, E, sigma, t):
    p = mk.params(SEED, n, E, sigma, matern_t=t)
    ref = _oracle_params(n, E, sigma, t)
    assert np.array_equal(p["S64"].cpu().numpy(), ref["S64"])
    assert np.array_equal(p["S"].cpu().numpy(), ref["S32"])
    # B, perm, G do not depend on the calibration
    assert np.array_equal(p["G"].cpu().numpy(), ref["G"])
    assert np.array_equal(p["perm"].cpu().numpy(), ref["perm"])


def test_matern_forward_matches_oracle(mk, orc):
    import torch

    x = workloads.mnist_uniform(64)
    phi = mk.forward(torch.from_numpy(x).cuda(), 1, SEED, 1.0, matern_t=40).cpu().numpy()
    ref, _, _ = orc.forward(x.astype(np.float64), 1, SEED, 1.0, p=_oracle_params(1024, 1, 1.0, 40))
    rel = np.linalg.norm(phi - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert rel.max() <= 1e-5


def test_matern_backward_runs_on_matern_plan(mk, orc):
    import torch

    x = workloads.mnist_uniform(16)
    dphi = workloads.grad_features(16, 2 * 1024)
    dx, dB, dG, dS = mk.backward(torch.from_numpy(x).cuda(), torch.from_numpy(dphi).cuda(), 1, SEED, 1.0,
                                 need_dx=True, need_params=True, matern_t=40)
    p = _oracle_params(1024, 1, 1.0, 40)
    ref = orc.backward(x.astype(np.float64), dphi.astype(np.float64), 1024, 1, p["B"], p["perm"], p["G"], p["S64"])
    for got, want in zip((dx, dB, dG, dS), ref):
        g = got.cpu().numpy().astype(np.float64).reshape(want.shape)
        assert np.linalg.norm(g - want) <= 1e-5 * np.linalg.norm(want)


def test_matern_plan_time_metric_size(mk):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = mk.params(7, 1024, 16, 1.0, matern_t=40)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("RBF-Matern plan n=1024 E=16 t=40: %.2f s" % dt)
    s = p["S64"].cpu().numpy()
    assert np.isfinite(s).all() and (s > 0).all()
    assert dt < 60


def test_matern_limits(mk):
    import torch

    with pytest.raises(mk.MckError):
        mk.params(1, 4096, 1, 1.0, matern_t=40)
    with pytest.raises(ValueError):
        mk.params(1, 16, 1, 1.0, matern_t=300)
    x = torch.zeros((2, 3000), device="cuda")
    with pytest.raises(mk.MckError):
        mk.forward(x, 1, 1, 1.0, matern_t=40)
