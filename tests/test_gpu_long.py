"""GPU parity for n > 2^15 (row pass over 2^15-element chunks plus column
passes over the high index bits) against the FP64 oracle.

Tolerances as for the single-pass path: integer transform inputs bit-exact,
float transform 1e-6 and FP32 features 1e-5 normwise per row; 16-bit phi
within its unit roundoff (2.5e-3 bfloat16, 3e-4 half)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mk():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_08159_amd as mk

    mk._lib.lib()
    return mk


def rowwise_rel(a, ref):
    a = np.asarray(a, np.float64).reshape(ref.shape)
    return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)


@pytest.mark.parametrize("m,batch", [(16, 3), (17, 2), (20, 2), (21, 1), (22, 1), (24, 1)])
def test_fwht_long_integer_bit_exact(mk, orc, m, batch):
    import torch

    n = 1 << m
    rng = np.random.default_rng(m)
    v = rng.integers(-1, 2, size=(batch, n)).astype(np.float32)
    got = mk.fwht(torch.from_numpy(v).cuda()).cpu().numpy()
    ref = orc.fwht(v.astype(np.float64))
    assert np.array_equal(got.astype(np.float64), ref)


@pytest.mark.parametrize("m", [16, 19, 23])
def test_fwht_long_float(mk, orc, m):
    import torch

    n = 1 << m
    v = workloads.normal(2, n, seed=m)
    got = mk.fwht(torch.from_numpy(v).cuda()).cpu().numpy()
    ref = orc.fwht(v.astype(np.float64))
    assert rowwise_rel(got, ref).max() <= 1e-6


@pytest.mark.parametrize("m", [16, 20, 24])
def test_long_params_bit_exact(mk, orc, m):
    # the generator at the largest sizes: 2^16 elements per norm lane at 2^24
    n = 1 << m
    p = mk.params(4242, n, 1, float(np.sqrt(n)))
    ref = orc.params(4242, n, 1, float(np.sqrt(n)))
    for k, r in (("B", "B"), ("perm", "perm"), ("G", "G"), ("S", "S32"), ("S64", "S64")):
        assert np.array_equal(p[k].cpu().numpy(), ref[r]), k


@pytest.mark.parametrize("d,E,batch", [(40000, 2, 3), (1 << 17, 1, 2), (70001, 3, 9), ((1 << 20) + 3, 1, 2),
                                       (1 << 24, 1, 1)])
def test_forward_long_matches_oracle(mk, orc, d, E, batch):
    import torch

    n = mk.padded_dim(d)
    sigma = float(np.sqrt(n))
    x = workloads.normal(batch, d, seed=d)
    phi = mk.forward(torch.from_numpy(x).cuda(), E, 4242, sigma).cpu().numpy()
    ref, _, _ = orc.forward(x.astype(np.float64), E, 4242, sigma)
    assert phi.shape == ref.shape
    assert rowwise_rel(phi, ref).max() <= 1e-5


def test_forward_long_unaligned_rows(mk, orc):
    import torch

    d, E, batch = 33000, 1, 3  # d not a multiple of 4: scalar loads
    x = workloads.normal(batch, d, seed=5)
    buf = torch.zeros(batch * d + 1, dtype=torch.float32, device="cuda")
    xv = buf[1:].view(batch, d)
    xv.copy_(torch.from_numpy(x).cuda())
    phi = mk.forward(xv, E, 9, 181.0).cpu().numpy()
    ref, _, _ = orc.forward(x.astype(np.float64), E, 9, 181.0)
    assert rowwise_rel(phi, ref).max() <= 1e-5


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
def test_long_vector_16bit_config(mk, orc, name):
    # batch 64 of N(0,1) inputs with n = 2^20, E = 4, sigma = sqrt(n), phi in
    # 16 bits; sampled rows against the oracle
    import torch

    dt = getattr(torch, name)
    n, E, batch = 1 << 20, 4, 64
    sigma = float(np.sqrt(n))
    x = workloads.normal(batch, n, seed=20)
    phi = mk.forward(torch.from_numpy(x).cuda(), E, workloads.FASTFOOD_SEED, sigma, out_dtype=dt)
    rows = [0, 31, 63]
    sub = phi[rows].float().cpu().numpy()
    ref, _, _ = orc.forward(x[rows].astype(np.float64), E, workloads.FASTFOOD_SEED, sigma)
    tol = {"bfloat16": 2.5e-3, "float16": 3e-4}[name]
    assert rowwise_rel(sub, ref).max() <= tol
    # and bit for bit the rounding of the FP32 path
    phi32 = mk.forward(torch.from_numpy(x[rows]).cuda(), E, workloads.FASTFOOD_SEED, sigma)
    assert torch.equal(phi32.to(dt), phi[rows])


def test_long_x16_input(mk, orc):
    import torch

    n, E = 1 << 16, 2
    x = torch.from_numpy(workloads.normal(4, n, seed=3)).cuda().to(torch.bfloat16)
    phi = mk.forward(x, E, 1, 256.0, out_dtype=torch.bfloat16)
    ref, _, _ = orc.forward(x.float().cpu().numpy().astype(np.float64), E, 1, 256.0)
    assert rowwise_rel(phi.float().cpu().numpy(), ref).max() <= 2.5e-3


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
def test_long_x16_ragged_input(mk, orc, name):
    # d not a multiple of 4: element-wise 16-bit loads in the first column pass
    import torch

    dt = getattr(torch, name)
    d, E = 40001, 2
    x = torch.from_numpy(workloads.normal(3, d, seed=4)).cuda().to(dt)
    phi = mk.forward(x, E, 3, 200.0, out_dtype=dt)
    ref, _, _ = orc.forward(x.float().cpu().numpy().astype(np.float64), E, 3, 200.0)
    tol = {"bfloat16": 2.5e-3, "float16": 3e-4}[name]
    assert rowwise_rel(phi.float().cpu().numpy(), ref).max() <= tol


def test_long_single_pass_only_calls_refuse(mk):
    import torch

    x = torch.zeros((2, 40000), device="cuda")
    with pytest.raises(mk.MckError):
        mk.project(x, 1, 1, 1.0)
    with pytest.raises(mk.MckError):
        mk.backward(x, torch.zeros((2, 2 * 65536), device="cuda"), 1, 1, 1.0)


def scale_rows(x, k):
    """Stored 16-bit-ready rows x 2^-k (exact), k per row."""
    return (x.astype(np.float64) * (2.0 ** -k.astype(np.float64))[:, None]).astype(np.float32)


@pytest.mark.parametrize("name", ["bfloat16", "float16"])
def test_long_vector_scaled_16bit_x_and_phi(mk, orc, name):
    # the long-vector reduced-precision configuration as stated: batch 64 of
    # N(0,1) rows, n = 2^20, E = 4, sigma = sqrt(n), x stored in 16 bits with
    # a per-row power-of-2 exponent (stored row max in [0.5, 1)), phi in 16
    # bits times 2^phi_exp.  Sampled rows against the oracle on the input
    # the stored values represent, and bit for bit the rounding of 2^j times
    # the FP32 map of that input.
    import torch

    dt = getattr(torch, name)
    n, E, batch = 1 << 20, 4, 64
    sigma = float(np.sqrt(n))
    x = workloads.normal(batch, n, seed=20)
    k = np.ceil(np.log2(np.abs(x).max(axis=1))).astype(np.int8)
    x16 = torch.from_numpy(scale_rows(x, k)).cuda().to(dt)
    ke = torch.from_numpy(k).cuda()
    phi, pexp = mk.forward_scaled(x16, E, workloads.FASTFOOD_SEED, sigma, x_exp=ke, out_dtype=dt)
    j = int(pexp[0].item())
    assert torch.equal(pexp, torch.full((batch,), j, dtype=torch.int8, device="cuda"))
    rows = [0, 31, 63]
    x_true = x16[rows].float().cpu().numpy().astype(np.float64) * (2.0 ** k[rows].astype(np.float64))[:, None]
    ref, _, _ = orc.forward(x_true, E, workloads.FASTFOOD_SEED, sigma)
    got = phi[rows].float().cpu().numpy().astype(np.float64) * 2.0 ** (-j)
    tol = {"bfloat16": 2.5e-3, "float16": 3e-4}[name]
    err = rowwise_rel(got, ref).max()
    print("%s x and phi, per-row exponents: max row error %.3e" % (name, err))
    assert err <= tol
    phi32 = mk.forward(torch.from_numpy(x_true.astype(np.float32)).cuda(), E, workloads.FASTFOOD_SEED, sigma)
    assert torch.equal((phi32.double() * 2.0 ** j).float().to(dt), phi[rows])


def test_long_vector_x_exponents_of_every_size(mk, orc):
    # rows of very different magnitude (2^-6 .. 2^7 times N(0,1)) carried in
    # half precision with their exponents, at a ragged d past 2^16
    import torch

    d, E, batch = 70001, 2, 8
    n = mk.padded_dim(d)
    sigma = float(np.sqrt(n))
    mag = np.array([-6, -2, 0, 3, 7, -1, 5, 1], np.int8)
    x = workloads.normal(batch, d, seed=31) * (2.0 ** mag.astype(np.float64))[:, None].astype(np.float32)
    k = np.ceil(np.log2(np.abs(x).max(axis=1))).astype(np.int8)
    x16 = torch.from_numpy(scale_rows(x, k)).cuda().to(torch.float16)
    phi, pexp = mk.forward_scaled(x16, E, 5, sigma, x_exp=torch.from_numpy(k).cuda(), out_dtype=torch.float16)
    j = int(pexp[0].item())
    x_true = x16.float().cpu().numpy().astype(np.float64) * (2.0 ** k.astype(np.float64))[:, None]
    ref, _, _ = orc.forward(x_true, E, 5, sigma)
    assert rowwise_rel(phi.float().cpu().numpy().astype(np.float64) * 2.0 ** (-j), ref).max() <= 3e-4


@pytest.mark.parametrize("d,E,batch", [(65536, 5, 37), (50000, 3, 300), (32769, 16, 9), (65533, 1, 1)])
def test_forward_2_16_one_block_rows(mk, orc, d, E, batch):
    # n = 2^16 runs the whole row in one block per (row, expansion): many
    # rows and expansions (several work items per block, partial row groups
    # per XCD), ragged d, d just past 2^15; sampled rows against the oracle
    import torch

    n = mk.padded_dim(d)
    assert n == 65536
    sigma = float(np.sqrt(n))
    x = workloads.normal(batch, d, seed=d + batch)
    phi = mk.forward(torch.from_numpy(x).cuda(), E, 77, sigma)
    rows = sorted({0, batch // 2, batch - 1, min(8, batch - 1), min(15, batch - 1)})
    got = phi[rows].cpu().numpy()
    ref, _, _ = orc.forward(x[rows].astype(np.float64), E, 77, sigma)
    assert rowwise_rel(got, ref).max() <= 1e-5


def test_forward_2_16_many_expansions(mk, orc):
    # E = 40 routings of Pi through the outer Benes stage (one colouring walk
    # per expansion at plan time); every row against the oracle
    import torch

    d, E, batch = 65536, 40, 5
    sigma = float(np.sqrt(d))
    x = workloads.normal(batch, d, seed=40)
    phi = mk.forward(torch.from_numpy(x).cuda(), E, 2024, sigma).cpu().numpy()
    ref, _, _ = orc.forward(x.astype(np.float64), E, 2024, sigma)
    assert rowwise_rel(phi, ref).max() <= 1e-5


def test_forward_2_16_every_row_unit_norm(mk):
    # ||phi(x)|| = 1 for every row (cos^2 + sin^2 per feature pair, scaled by
    # 1 / sqrt(nE)): a row or expansion that no work item wrote shows here
    import torch

    d, E, batch = 60000, 3, 600
    x = torch.from_numpy(workloads.normal(batch, d, seed=6)).cuda()
    phi = mk.forward(x, E, 8, 256.0)
    norms = torch.linalg.vector_norm(phi.double(), dim=1).cpu().numpy()
    assert np.abs(norms - 1.0).max() <= 1e-5
