"""16-bit storage of x and phi (bfloat16, IEEE half) with FP32 arithmetic.

Checks, through the C ABI:
  * consistency: phi stored in 16 bits is exactly the round-to-nearest-even
    of the FP32 path's phi (same arithmetic, only the final rounding differs);
  * parity with the FP64 oracle within the storage format's unit roundoff
    (normwise per row: 2.5e-3 for bfloat16, u = 2^-9; 3e-4 for half,
    u = 2^-12), on x given in FP32 or in the 16-bit type itself (oracle fed
    the exactly widened values);
  * unsupported storage pairs are refused.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = {"bfloat16": 2.5e-3, "float16": 3e-4}


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
    den = np.linalg.norm(ref, axis=1)
    den[den == 0] = 1.0
    return np.linalg.norm(a - ref, axis=1) / den


def bf16_rne(f32):
    """float32 -> bfloat16 bits, round to nearest even (finite inputs)."""
    u = np.asarray(f32, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def to_f64(torch, t):
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
@pytest.mark.parametrize("d,E,batch", [(784, 4, 37), (13, 2, 9), (1024, 1, 5), (4096, 2, 3), (12000, 2, 3),
                                         (16384, 1, 2), (20000, 2, 3), (32768, 1, 2)])
def test_phi16_is_rounded_fp32_phi(mk, name, d, E, batch):
    import torch

    dt = getattr(torch, name)
    x = torch.from_numpy(workloads.normal(batch, d, seed=d)).cuda()
    sigma = float(np.sqrt(mk.padded_dim(d)))
    phi32 = mk.forward(x, E, 11, sigma).cpu().numpy()
    phi16 = mk.forward(x, E, 11, sigma, out_dtype=dt).cpu()
    if name == "float16":
        expect = phi32.astype(np.float16).view(np.uint16)
        got = phi16.numpy().view(np.uint16)
    else:
        expect = bf16_rne(phi32)
        got = phi16.view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
@pytest.mark.parametrize("x16", [False, True])
def test_phi16_matches_oracle(mk, orc, name, x16):
    import torch

    dt = getattr(torch, name)
    x = workloads.mnist_sparse(64)
    xt = torch.from_numpy(x).cuda()
    if x16:
        xt = xt.to(dt)
        x = xt.float().cpu().numpy()
    phi = mk.forward(xt, 16, workloads.FASTFOOD_SEED, 2.0, out_dtype=dt)
    assert phi.dtype == dt
    ref, _, _ = orc.forward(x.astype(np.float64), 16, workloads.FASTFOOD_SEED, 2.0)
    assert rowwise_rel(to_f64(torch, phi), ref).max() <= TOL[name]


def test_unsupported_pairs_refused(mk):
    import torch

    x = torch.zeros((2, 8), device="cuda", dtype=torch.bfloat16)
    with pytest.raises(mk.MckError):
        mk.forward(x, 1, 1, 1.0, out_dtype=torch.float32)
    with pytest.raises(mk.MckError):
        mk.forward(x, 1, 1, 1.0, out_dtype=torch.float16)


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
@pytest.mark.parametrize("d", [9000, 16384, 30000])
def test_phi16_large_rows_match_oracle(mk, orc, name, d):
    # rows of 2^14 and 2^15 (packed parameters, 32 values per lane) with
    # 16-bit x and 16-bit phi
    import torch

    dt = getattr(torch, name)
    n = mk.padded_dim(d)
    xt = torch.from_numpy(workloads.normal(3, d, seed=d)).cuda().to(dt)
    x = xt.float().cpu().numpy()
    sigma = float(np.sqrt(n))
    phi = mk.forward(xt, 2, 13, sigma, out_dtype=dt)
    ref, _, _ = orc.forward(x.astype(np.float64), 2, 13, sigma)
    assert rowwise_rel(to_f64(torch, phi), ref).max() <= TOL[name]
