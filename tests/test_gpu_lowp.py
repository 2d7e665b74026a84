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


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
@pytest.mark.parametrize("d,E", [(784, 16), (13, 2), (5000, 4), (30000, 2)])
def test_scaled_storage_matches_oracle(mk, orc, name, d, E):
    # per-row power-of-2 scaling: x rows of very different magnitude carried
    # in 16 bits with their exponents, phi stored times 2^phi_exp
    import torch

    dt = getattr(torch, name)
    batch = 6
    n = mk.padded_dim(d)
    sigma = float(np.sqrt(n))
    base = workloads.normal(batch, d, seed=d + 1)
    k = np.array([-3, 0, 2, -1, 1, 0][:batch], np.int8)
    x16 = torch.from_numpy(base).cuda().to(dt)
    phi, pexp = mk.forward_scaled(x16, E, 9, sigma, x_exp=torch.from_numpy(k).cuda(), out_dtype=dt)
    j = int(pexp[0].item())
    assert torch.equal(pexp, torch.full((batch,), j, dtype=torch.int8, device="cuda"))
    assert 1.0 / np.sqrt(n * E) * 2.0 ** j <= 1.0 < 1.0 / np.sqrt(n * E) * 2.0 ** (j + 1)
    x_true = x16.float().cpu().numpy().astype(np.float64) * (2.0 ** k.astype(np.float64))[:, None]
    ref, _, _ = orc.forward(x_true, E, 9, sigma)
    got = to_f64(torch, phi) * 2.0 ** (-j)
    assert rowwise_rel(got, ref).max() <= TOL[name]


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
def test_scaled_phi_is_rounded_scaled_fp32_phi(mk, name):
    import torch

    dt = getattr(torch, name)
    x = torch.from_numpy(workloads.normal(7, 1000, seed=4)).cuda()
    E, sigma = 8, 32.0
    phi32 = mk.forward(x, E, 3, sigma).cpu().numpy()
    phi16, pexp = mk.forward_scaled(x, E, 3, sigma, out_dtype=dt)
    j = int(pexp[0].item())
    scaled = (phi32.astype(np.float64) * 2.0 ** j).astype(np.float32)  # exact: a power of two
    if name == "float16":
        assert np.array_equal(phi16.cpu().numpy().view(np.uint16), scaled.astype(np.float16).view(np.uint16))
    else:
        assert np.array_equal(phi16.cpu().view(torch.int16).numpy().view(np.uint16), bf16_rne(scaled))
    # FP32 storage: exactly 2^j times the plain map
    phif, _ = mk.forward_scaled(x, E, 3, sigma)
    assert np.array_equal(phif.cpu().numpy(), scaled)


def test_scaled_half_beats_plain_half_when_features_are_small(mk, orc):
    # n = 8192, E = 16: c = 2^-8.5, so plain half phi has many subnormal
    # features; the scaled form keeps them normal
    import torch

    x = torch.from_numpy(workloads.normal(4, 8192, seed=8)).cuda()
    sigma = float(np.sqrt(8192))
    ref, _, _ = orc.forward(x.cpu().numpy().astype(np.float64), 16, 21, sigma)
    plain = to_f64(torch, mk.forward(x, 16, 21, sigma, out_dtype=torch.float16))
    sc, pexp = mk.forward_scaled(x, 16, 21, sigma, out_dtype=torch.float16)
    scaled = to_f64(torch, sc) * 2.0 ** (-int(pexp[0].item()))
    e_plain, e_scaled = rowwise_rel(plain, ref).max(), rowwise_rel(scaled, ref).max()
    assert e_scaled <= e_plain and e_scaled <= TOL["float16"]


def test_scaled_long_rows(mk, orc):
    # n = 2^16 (the multi-pass path): phi scaled by 2^j, bit for bit the
    # rounding of 2^j times the FP32 map, and within the half bound
    import torch

    x = torch.from_numpy(workloads.normal(3, 40000, seed=5)).cuda()
    sigma = 256.0
    phi32 = mk.forward(x, 2, 17, sigma).cpu().numpy()
    sc, pexp = mk.forward_scaled(x, 2, 17, sigma, out_dtype=torch.float16)
    j = int(pexp[0].item())
    scaled = (phi32.astype(np.float64) * 2.0 ** j).astype(np.float32)
    assert np.array_equal(sc.cpu().numpy().view(np.uint16), scaled.astype(np.float16).view(np.uint16))
    ref, _, _ = orc.forward(x.cpu().numpy().astype(np.float64), 2, 17, sigma)
    assert rowwise_rel(to_f64(torch, sc) * 2.0 ** (-j), ref).max() <= TOL["float16"]


def test_scaled_refusals(mk):
    import torch

    xb = torch.zeros((2, 8), device="cuda", dtype=torch.bfloat16)
    with pytest.raises(mk.MckError, match="UNSUPPORTED"):
        mk.forward_scaled(xb, 1, 1, 1.0, out_dtype=torch.float16)
