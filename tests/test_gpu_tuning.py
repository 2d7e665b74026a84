"""Forward launch choices and the autotuner.

Every compiled register split and grid target must compute the map of
equation "mckernel" (section "McKernel"): phi and z within 1e-5 per row of
the FP64 oracle, 16-bit phi the round-to-nearest-even of the FP32 phi of the
same split, the batched call equal to the plain call under the same choice
bit for bit, the explicit-parameter forward within 1e-5 of the oracle.  The
autotuner stores a valid choice per n, and the batched call replays from a
HIP graph."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
TUNABLE = [1 << m for m in range(9, 15)]  # both splits compiled
WAVES = (2048, 4096, 8192, 16384, 32768, 65536)


@pytest.fixture(scope="module")
def mk():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_08159_amd as mk

    mk._lib.lib()
    return mk


@pytest.fixture(autouse=True)
def restore_defaults(mk):
    yield
    for m in range(1, 16):
        mk.set_forward_tuning(1 << m)


def rowwise_rel(a, ref):
    den = np.linalg.norm(ref, axis=1)
    den[den == 0] = 1.0
    return np.linalg.norm(a - ref, axis=1) / den


def bf16_rne(f32):
    u = np.asarray(f32, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def test_defaults(mk):
    for m in range(1, 16):
        assert mk.forward_tuning(1 << m) == ((5 if m >= 13 else 4), 16384)


def test_set_is_validated(mk):
    with pytest.raises(mk.MckError, match="UNSUPPORTED"):
        mk.set_forward_tuning(256, split=5)  # one split below 2^9
    with pytest.raises(mk.MckError, match="UNSUPPORTED"):
        mk.set_forward_tuning(32768, split=4)
    with pytest.raises(mk.MckError, match="INVALID"):
        mk.set_forward_tuning(1024, waves=10)
    with pytest.raises(mk.MckError, match="INVALID"):
        mk.set_forward_tuning(1000, split=4)
    with pytest.raises(mk.MckError, match="INVALID"):
        mk.set_forward_tuning(65536, split=5)
    mk.set_forward_tuning(1024, split=5, waves=4096)
    assert mk.forward_tuning(1024) == (5, 4096)
    mk.set_forward_tuning(1024)
    assert mk.forward_tuning(1024) == (4, 16384)


@pytest.mark.parametrize("n", TUNABLE)
@pytest.mark.parametrize("split", [4, 5])
def test_every_split_matches_oracle(mk, orc, n, split):
    import torch

    # ragged d (no vector path) and d = n (vector path), E = 3, several rows
    E, seed, sigma = 3, 77, float(np.sqrt(n))
    for d, batch in ((n - 3, 5), (n, 4)):
        x = workloads.normal(batch, d, seed=d + split)
        xt = torch.from_numpy(x).cuda()
        ref_phi, ref_z, p = orc.forward(x.astype(np.float64), E, seed, sigma)
        mk.set_forward_tuning(n, split=split, waves=2048)
        phi = mk.forward(xt, E, seed, sigma)
        z = mk.project(xt, E, seed, sigma)
        mk.set_forward_tuning(n, split=split, waves=65536)
        phi_w = mk.forward(xt, E, seed, sigma)
        assert rowwise_rel(phi.cpu().numpy().astype(np.float64), ref_phi).max() <= TOL
        assert rowwise_rel(z.cpu().numpy().astype(np.float64), ref_z).max() <= TOL
        # the grid target changes the chunking of the expansions, not the arithmetic
        assert torch.equal(phi, phi_w)


@pytest.mark.parametrize("n", [512, 4096, 16384])
@pytest.mark.parametrize("split", [4, 5])
def test_split_16bit_and_explicit_forms(mk, orc, n, split):
    import torch

    E, seed, sigma = 2, 5, float(np.sqrt(n))
    xh = workloads.normal(6, n, seed=n)
    x = torch.from_numpy(xh).cuda()
    mk.set_forward_tuning(n, split=split)
    phi32 = mk.forward(x, E, seed, sigma)
    bf = mk.forward(x, E, seed, sigma, out_dtype=torch.bfloat16).cpu()
    hf = mk.forward(x, E, seed, sigma, out_dtype=torch.float16).cpu()
    p32 = phi32.cpu().numpy()
    assert np.array_equal(bf.view(torch.int16).numpy().view(np.uint16), bf16_rne(p32))
    assert np.array_equal(hf.numpy().view(np.uint16), p32.astype(np.float16).view(np.uint16))
    p = mk.params(seed, n, E, sigma)
    phi_p = mk.forward_p(x, p["B"], p["perm"], p["G"], p["S"])
    ref, _, _ = orc.forward(xh.astype(np.float64), E, seed, sigma)
    assert rowwise_rel(phi_p.cpu().numpy().astype(np.float64), ref).max() <= TOL
    got = mk.forward_batched([(x, E, seed, sigma), (x[:2], 1, seed + 1, sigma)])
    assert torch.equal(got[0], phi32)
    assert torch.equal(got[1], mk.forward(x[:2], 1, seed + 1, sigma))


def _maps(count, seed, max_batch, max_E, m_lo, m_hi):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        m = int(rng.integers(m_lo, m_hi + 1))
        batch = int(rng.integers(1, max_batch + 1))
        E = int(rng.integers(1, max_E + 1))
        d = int(rng.integers((1 << m) // 2 + 1, (1 << m) + 1))
        out.append((workloads.normal(batch, d, seed=100 + k), E, 2000 + k, float(np.sqrt(1 << m))))
    return out


def test_autotune_batched(mk, orc):
    import torch

    maps = _maps(14, 3, max_batch=96, max_E=4, m_lo=6, m_hi=15)
    dev = [(torch.from_numpy(x).cuda(), E, s, sg) for x, E, s, sg in maps]
    chosen = mk.autotune_batched(dev, reps=2)
    ns = sorted({mk.padded_dim(x.shape[1]) for x, _, _, _ in maps})
    assert sorted(chosen) == ns
    for n, (split, waves) in chosen.items():
        m = n.bit_length() - 1
        allowed = (4, 5) if 9 <= m <= 14 else ((5,) if m >= 14 else (4,))
        assert split in allowed, (n, split)
        assert waves in WAVES, (n, waves)
        assert mk.forward_tuning(n) == (split, waves)
    got = mk.forward_batched(dev)
    for (x, E, s, sg), phi in zip(dev, got):
        assert torch.equal(phi, mk.forward(x, E, s, sg))
    for k in (0, 5, 11):
        x, E, s, sg = maps[k]
        ref, _, _ = orc.forward(x.astype(np.float64), E, s, sg)
        assert rowwise_rel(got[k].cpu().numpy().astype(np.float64), ref).max() <= TOL


def test_autotune_refused_under_capture(mk):
    import torch

    x = torch.from_numpy(workloads.normal(4, 1000, seed=1)).cuda()
    mk.forward(x, 2, 3, 30.0)  # plan cached
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(mk.MckError, match="graph capture"):
        with torch.cuda.graph(g):
            mk.autotune_batched([(x, 2, 3, 30.0)], reps=1)
    torch.cuda.synchronize()


def test_batched_graph_replays_match_eager(mk):
    import torch

    maps = _maps(10, 4, max_batch=64, max_E=4, m_lo=4, m_hi=15)
    dev = [(torch.from_numpy(x).cuda(), E, s, sg) for x, E, s, sg in maps]
    ref = [p.clone() for p in mk.forward_batched(dev)]  # builds and caches the plans
    outs = [torch.empty_like(r) for r in ref]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mk.forward_batched(dev, outs=outs)
    for k in range(4):
        for o in outs:
            o.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), k
        junk = mk.forward(dev[0][0][:3], 2, 9, 1.0)  # eager work between replays
        torch.cuda.synchronize()
        del junk
