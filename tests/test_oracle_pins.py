"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics,
independent of the oracle's own code (CPU only).

Each test names what it pins and where the fact comes from.
"""
import math
import os
import struct

import numpy as np
import pytest
import scipy.linalg
import scipy.stats as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ FWHT (P1)
def _load_golden_matrix(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(t) for t in line.split()])
    return np.array(rows, dtype=np.float64)


def test_fwht_matches_paper_recursion_fixture(orc):
    # H_3 written out by hand from the recursion of section "Fast Walsh Hadamard".
    H8 = _load_golden_matrix("sylvester_h8.txt")
    assert H8.shape == (8, 8)
    cols = orc.fwht(np.eye(8))  # row k = H e_k = column k of H
    np.testing.assert_array_equal(cols.T, H8)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
def test_fwht_dense_scipy_hadamard(orc, n):
    # scipy.linalg.hadamard builds the Sylvester matrix in natural order.
    rng = np.random.default_rng(n)
    v = rng.integers(-50, 51, size=(5, n)).astype(np.float64)
    ref = v @ scipy.linalg.hadamard(n).T.astype(np.float64)
    np.testing.assert_array_equal(orc.fwht(v), ref)


@pytest.mark.parametrize("m", [7, 9, 12])
def test_fwht_popcount_closed_form(orc, m):
    # (H v)_i = sum_k (-1)^popcount(i & k) v_k, by induction on the top bit of
    # the recursion H_k = [[H, H], [H, -H]].  Exact on integer input.
    n = 1 << m
    idx = np.arange(n, dtype=np.uint32)
    andm = idx[:, None] & idx[None, :]
    par = np.zeros_like(andm)
    x = andm.copy()
    while x.any():
        par ^= x & 1
        x >>= 1
    H = (1 - 2 * par.astype(np.int64)).astype(np.float64)
    rng = np.random.default_rng(m)
    v = rng.integers(-8, 9, size=(2, n)).astype(np.float64)
    np.testing.assert_array_equal(orc.fwht(v), v @ H.T)


@pytest.mark.parametrize("n", [2, 16, 1024, 1 << 15])
def test_fwht_involution_and_basis(orc, n):
    # H H = n I, H e_0 = 1, H 1 = n e_0.
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3, n))
    hh = orc.fwht(orc.fwht(v))
    np.testing.assert_allclose(hh, n * v, rtol=0, atol=1e-12 * n * np.abs(v).max() * math.log2(n) + 1e-300)
    e0 = np.zeros(n); e0[0] = 1
    np.testing.assert_array_equal(orc.fwht(e0), np.ones(n))
    np.testing.assert_array_equal(orc.fwht(np.ones(n)), n * e0)


# ------------------------------------------------------------------ hash (P8)
def test_murmur3_matches_sklearn(orc):
    from sklearn.utils import murmurhash3_32

    rng = np.random.default_rng(7)
    for length in range(0, 24):
        for _ in range(8):
            key = bytes(rng.integers(0, 256, size=length, dtype=np.uint8))
            seed = int(rng.integers(0, 2**32))
            assert orc.murmur3(key, seed) == murmurhash3_32(key, seed=seed, positive=True)


def test_hash4_is_murmur_of_le_key(orc):
    from sklearn.utils import murmurhash3_32

    rng = np.random.default_rng(8)
    for _ in range(200):
        w = [int(t) for t in rng.integers(0, 2**32, size=4)]
        seed = int(rng.integers(0, 2**32))
        key = struct.pack("<4I", *w)
        assert orc.hash4(seed, *w) == murmurhash3_32(key, seed=seed, positive=True)
    # the paper's experiment seed
    key = struct.pack("<4I", 2, 5, 17, 1)
    assert orc.hash4(1398239763, 2, 5, 17, 1) == murmurhash3_32(key, seed=1398239763, positive=True)


# ------------------------------------------------------------------ elementary functions
def test_ln32_error_bound(orc):
    # u = k 2^-24 (the Box-Muller radius input) over a stride of all k, plus
    # general floats; bound: 3 ulp of the result against FP64 log.
    ks = np.concatenate([np.arange(1, 4097), np.arange(4097, 2**24 + 1, 104729), [2**24 - 1, 2**24]])
    us = np.concatenate([ks * 2.0**-24, np.random.default_rng(0).random(2000) * 100 + 1e-30])
    us = us.astype(np.float32)
    got = np.array([orc.ln32(u) for u in us], dtype=np.float64)
    ref = np.log(us.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    ulp[ref == 0] = np.spacing(np.float32(1))
    assert np.max(np.abs(got - ref) / ulp) <= 3.0
    assert orc.ln32(1.0) == 0.0


def test_sincos2pi32_error_bound(orc):
    ks = np.concatenate([np.arange(0, 2**24, 40009), np.arange(0, 4096), 2**22 * np.arange(4) + 1,
                         2**21 * np.arange(8), 2**21 * np.arange(8) - 1])
    ks = ks[(ks >= 0) & (ks < 2**24)]
    for k in ks:
        c, s = orc.sincos2pi32(int(k))
        a = 2 * np.pi * np.longdouble(int(k)) / 2**24
        assert abs(float(c) - float(np.cos(a))) <= 2.5e-7
        assert abs(float(s) - float(np.sin(a))) <= 2.5e-7
        assert abs(float(c) ** 2 + float(s) ** 2 - 1.0) <= 1e-6


def test_ln64_error_bound(orc):
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.random(20000) + 1e-300, rng.random(2000) * 1e6,
                        np.exp(rng.uniform(-700, 700, 2000)), (rng.integers(0, 2**32, 2000) + 1.0) * 2.0**-32])
    got = np.array([orc.ln64(x) for x in v])
    ref = np.log(v.astype(np.longdouble))
    err = np.abs(got.astype(np.longdouble) - ref).astype(np.float64)
    ulp = np.spacing(np.abs(ref.astype(np.float64)))
    ulp[ref == 0] = np.spacing(1.0)
    assert np.max(err / ulp) <= 3.0
    assert orc.ln64(1.0) == 0.0


def test_cos2pi64_error_bound(orc):
    hs = np.concatenate([np.random.default_rng(4).integers(0, 2**32, 20000),
                         2**30 * np.arange(4), 2**29 * np.arange(8), 2**29 * np.arange(1, 8) - 1])
    got = np.array([orc.cos2pi64(int(h)) for h in hs])
    ref = np.cos(2 * np.pi * hs.astype(np.longdouble) / 2**32).astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-15


# ------------------------------------------------------------------ Box-Muller (P10)
def test_boxmuller_closed_cases(orc):
    top = (2**24 - 1) << 8          # (a>>8)+1 = 2^24  ->  u1 = 1  ->  r = 0
    g0, g1 = orc.boxmuller32(top, 12345 << 8)
    assert g0 == 0.0 and g1 == 0.0
    a = 99 << 8                      # u1 = 100 / 2^24
    r = math.sqrt(-2.0 * math.log(100 * 2.0**-24))
    g0, g1 = orc.boxmuller32(a, 0)   # angle 0  ->  (r, 0)
    assert abs(float(g0) - r) <= 3e-7 * r and g1 == 0.0
    g0, g1 = orc.boxmuller32(a, (1 << 22) << 8)  # quarter turn -> (0, r)
    assert g0 == 0.0 and abs(float(g1) - r) <= 3e-7 * r
    g0, g1 = orc.boxmuller32(a, (1 << 23) << 8)  # half turn -> (-r, 0)
    assert abs(float(g0) + r) <= 3e-7 * r and g1 == 0.0


def test_boxmuller_matches_libm_formula(orc):
    rng = np.random.default_rng(11)
    for a, b in rng.integers(0, 2**32, size=(3000, 2)):
        g0, g1 = orc.boxmuller32(int(a), int(b))
        u1 = ((int(a) >> 8) + 1) * 2.0**-24
        ang = 2 * math.pi * (int(b) >> 8) * 2.0**-24
        r = math.sqrt(-2 * math.log(u1))
        assert abs(float(g0) - r * math.cos(ang)) <= 1e-6 * (1 + r)
        assert abs(float(g1) - r * math.sin(ang)) <= 1e-6 * (1 + r)


# ------------------------------------------------------------------ distributions (P9)
def test_B_is_balanced_rademacher(orc):
    p = orc.params(1398239763, 4096, 8, 1.0)
    B = p["B"]
    assert set(np.unique(B)) == {-1.0, 1.0}
    k = int((B < 0).sum())
    assert st.binomtest(k, B.size, 0.5).pvalue > 1e-4
    # neighbouring entries uncorrelated
    assert abs(np.mean(B[:, 1:] * B[:, :-1])) < 4 / math.sqrt(B.size)


def test_perm_is_bijection_and_uniform(orc):
    for n in (2, 8, 1024):
        P = orc.params(5, n, 3, 1.0)["perm"]
        for e in range(3):
            assert sorted(P[e].tolist()) == list(range(n))
    # n = 4: all 24 permutations equally likely (chi-square over seeds x expansions)
    counts = {}
    for seed in range(1500):
        P = orc.params(seed, 4, 16, 1.0)["perm"]
        for row in P:
            counts[tuple(row)] = counts.get(tuple(row), 0) + 1
    assert len(counts) == 24
    obs = np.array(list(counts.values()), dtype=np.float64)
    assert st.chisquare(obs).pvalue > 1e-4


def test_G_is_standard_normal(orc):
    G = orc.params(1398239763, 4096, 8, 1.0)["G"].astype(np.float64).ravel()
    assert st.kstest(G, "norm").pvalue > 1e-4
    assert abs(G.mean()) < 4 / math.sqrt(G.size)
    assert abs(G.var() - 1) < 4 * math.sqrt(2 / G.size)


@pytest.mark.parametrize("n", [2, 16, 1024])
def test_chi_radius_distribution(orc, n):
    E = max(1, 8192 // n)
    p = orc.params(424242, n, E, 1.0, with_aux=True)
    s = p["chi"].ravel()
    dist = st.chi(n)
    assert st.kstest(s, dist.cdf).pvalue > 1e-4
    assert abs(s.mean() - dist.mean()) < 5 * dist.std() / math.sqrt(s.size)


def test_chi_mean_at_1024():
    # the value quoted for the FP32 metric configuration: E[chi(1024)]
    assert abs(st.chi(1024).mean() - 31.99219) < 1e-4


# ------------------------------------------------------------------ composition (P2, P3, P4)
def _dense_Z(p, n, e, S):
    H = scipy.linalg.hadamard(n).astype(np.float64)
    Pm = np.zeros((n, n))
    Pm[np.arange(n), p["perm"][e]] = 1.0
    return (np.diag(S[e]) @ H @ np.diag(p["G"][e].astype(np.float64)) @ Pm @ H
            @ np.diag(p["B"][e].astype(np.float64)))


@pytest.mark.parametrize("n", [2, 4, 16, 64])
def test_dense_product_equals_fast_path(orc, n):
    # P4: Z = S H G Pi H B multiplied out densely for n <= 64.
    E = 3
    p = orc.params(77, n, E, 1.7)
    rng = np.random.default_rng(n)
    d = max(1, n - n // 4)
    x = rng.standard_normal((4, d))
    z = orc.project(x, n, E, p["B"], p["perm"], p["G"], p["S64"])
    xh = np.zeros((4, n)); xh[:, :d] = x
    for e in range(E):
        ref = xh @ _dense_Z(p, n, e, p["S64"]).T
        np.testing.assert_allclose(z[:, e * n:(e + 1) * n], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("n,sigma", [(16, 1.0), (64, 2.5), (256, 0.3)])
def test_row_norm_identity(orc, n, sigma):
    # P2: H B B H = n I and Pi orthogonal give Z Z^T = n S H G^2 H S, whose
    # diagonal is s_j^2 / sigma^2 exactly (the chi radius over sigma).
    E = 2
    p = orc.params(31337, n, E, sigma, with_aux=True)
    Z = orc.project(np.eye(n), n, E, p["B"], p["perm"], p["G"], p["S64"])  # row k = Z e_k
    H = scipy.linalg.hadamard(n).astype(np.float64)
    for e in range(E):
        Ze = Z[:, e * n:(e + 1) * n].T
        ZZ = Ze @ Ze.T
        np.testing.assert_allclose(np.diag(ZZ), p["chi"][e] ** 2 / sigma**2, rtol=1e-12)
        S = np.diag(p["S64"][e])
        G2 = np.diag(p["G"][e].astype(np.float64) ** 2)
        np.testing.assert_allclose(ZZ, n * S @ H @ G2 @ H @ S, rtol=0, atol=1e-12 * np.abs(ZZ).max())


def test_special_case_identity_parameters(orc):
    # P3: B = 1, Pi = id, G = 1  ->  z = S (H H xhat) = n S xhat.
    n, E, d = 32, 2, 27
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, d))
    S = rng.standard_normal((E, n))
    z = orc.project(x, n, E, np.ones((E, n)), np.tile(np.arange(n, dtype=np.int32), (E, 1)),
                    np.ones((E, n)), S)
    xh = np.zeros((3, n)); xh[:, :d] = x
    for e in range(E):
        ref = n * S[e] * xh
        np.testing.assert_allclose(z[:, e * n:(e + 1) * n], ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())


def test_S_normalisation_formula(orc):
    # S'_j = s_j / (sigma sqrt(n) ||G||_F), S32 = RNE(S64)
    n, E, sigma = 128, 2, 1.3
    p = orc.params(9, n, E, sigma, with_aux=True)
    G64 = p["G"].astype(np.float64)
    np.testing.assert_allclose(p["norm2"], (G64**2).sum(axis=1), rtol=1e-14)
    ref = p["chi"] / (sigma * math.sqrt(n) * np.sqrt(p["norm2"]))[:, None]
    np.testing.assert_allclose(p["S64"], ref, rtol=1e-15)
    np.testing.assert_array_equal(p["S32"], p["S64"].astype(np.float32))


# ------------------------------------------------------------------ feature map (P5, P6, P7, P12)
def test_feature_norm_and_cos_difference(orc):
    # ||phi|| = 1, and phi(x).phi(y) = mean_j cos(z_j(x) - z_j(y)).
    n, E = 64, 4
    rng = np.random.default_rng(12)
    x = rng.standard_normal((2, 50))
    phi, z, _ = orc.forward(x, E, 2024, 3.0)
    assert phi.shape == (2, 2 * n * E)
    np.testing.assert_allclose(np.linalg.norm(phi, axis=1), 1.0, rtol=1e-13)
    np.testing.assert_allclose(phi[0] @ phi[1], np.mean(np.cos(z[0] - z[1])), rtol=1e-12)


def test_feature_layout_cos_then_sin(orc):
    n, E = 8, 3
    x = np.random.default_rng(2).standard_normal((1, 8))
    phi, z, _ = orc.forward(x, E, 1, 1.0)
    c = 1 / math.sqrt(n * E)
    np.testing.assert_allclose(phi[0, :n * E], c * np.cos(z[0]), rtol=1e-15)
    np.testing.assert_allclose(phi[0, n * E:], c * np.sin(z[0]), rtol=1e-15)


def test_kernel_unbiased_over_seeds(orc):
    # P6: each row of Z is N(0, sigma^-2 I) (uniform direction, chi(n)/sigma
    # norm), so E_seed[phi(x).phi(y)] = exp(-||x-y||^2 / (2 sigma^2)).
    n, sigma, seeds = 16, 1.0, 600
    rng = np.random.default_rng(21)
    x = rng.standard_normal(n)
    u = rng.standard_normal(n); u /= np.linalg.norm(u)
    for r in (0.5, 1.0, 2.0):
        y = x + r * u
        vals = []
        for s in range(seeds):
            phi, _, _ = orc.forward(np.stack([x, y]), 1, 1000 + s, sigma)
            vals.append(phi[0] @ phi[1])
        vals = np.array(vals)
        k = math.exp(-r * r / (2 * sigma**2))
        se = vals.std(ddof=1) / math.sqrt(seeds)
        assert abs(vals.mean() - k) < 4 * se + 1e-3


def test_kernel_error_shrinks_with_E(orc):
    # P7: |phi(x).phi(y) - k(x,y)| shrinks roughly like 1/sqrt(nE).
    n, sigma = 64, 4.0
    rng = np.random.default_rng(22)
    pairs = [(rng.standard_normal(n), rng.standard_normal(n)) for _ in range(6)]
    rms = {}
    for E in (1, 4, 16, 64):
        errs = []
        for i, (x, y) in enumerate(pairs):
            for s in range(4):
                phi, _, _ = orc.forward(np.stack([x, y]), E, 50 * i + s, sigma)
                k = math.exp(-np.sum((x - y) ** 2) / (2 * sigma**2))
                errs.append(phi[0] @ phi[1] - k)
        rms[E] = math.sqrt(np.mean(np.square(errs)))
    assert rms[64] < rms[1] / 3
    assert rms[16] < rms[1] / 1.5
    scaled = [rms[E] * math.sqrt(n * E) for E in rms]
    assert max(scaled) / min(scaled) < 4


def test_parameter_count_from_paper(orc):
    # P12: C (2 [S]_2 E + 1) learned parameters => 2 n E features per sample.
    for line in open(os.path.join(GOLDEN, "parameter_count.txt")):
        if line.startswith("#") or not line.strip():
            continue
        C, S, E, expected = (int(t) for t in line.split())
        phi, _, _ = orc.forward(np.zeros((1, S)), E, 3, 1.0)
        assert C * (phi.shape[1] + 1) == expected


def test_padded_dim(orc):
    assert [orc.padded_dim(d) for d in (1, 2, 3, 4, 5, 784, 1024, 1025)] == [2, 2, 4, 4, 8, 1024, 1024, 2048]


# ------------------------------------------------------------------ adjoint (P11)
def _loss_and_grads(orc, x, dphi, n, E, B, perm, G, S):
    z = orc.project(x, n, E, B, perm, G, S)
    phi = orc.features(z, n, E)
    return float(np.sum(phi * dphi)), orc.backward(x, dphi, n, E, B, perm, G, S)


def test_adjoint_dot_product(orc):
    # <Z x, u> = <x, Z^T u> for the linear part: with phi's cotangent chosen as
    # dphi = c^-1 [-sin z * u, cos z * u] the backward returns Z^T u exactly.
    n, E, d = 32, 3, 29
    p = orc.params(8, n, E, 1.1)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, d))
    u = rng.standard_normal((2, n * E))
    z = orc.project(x, n, E, p["B"], p["perm"], p["G"], p["S64"])
    c = 1 / math.sqrt(n * E)
    dphi = np.concatenate([-np.sin(z) * u, np.cos(z) * u], axis=1) / c
    dx, _, _, _ = orc.backward(x, dphi, n, E, p["B"], p["perm"], p["G"], p["S64"])
    lhs = np.sum(z * u, axis=1)
    rhs = np.sum(x * dx, axis=1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10)


def test_adjoint_central_differences(orc):
    n, E, d = 16, 2, 13
    p = orc.params(15, n, E, 1.0)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, d))
    B = p["B"].astype(np.float64) * (1 + 0.1 * rng.standard_normal((E, n)))
    G = p["G"].astype(np.float64)
    S = p["S64"].copy()
    dphi = rng.standard_normal((2, 2 * n * E))
    _, (dx, dB, dG, dS) = _loss_and_grads(orc, x, dphi, n, E, B, p["perm"], G, S)
    h = 1e-3

    def fd(arr, idx, setter):
        a1 = arr.copy(); a1[idx] += h
        a2 = arr.copy(); a2[idx] -= h
        return (setter(a1) - setter(a2)) / (2 * h)

    L = lambda xx, BB, GG, SS: _loss_and_grads(orc, xx, dphi, n, E, BB, p["perm"], GG, SS)[0]
    for idx in [(0, 0), (1, 5), (0, d - 1)]:
        g = fd(x, idx, lambda a: L(a, B, G, S))
        assert abs(g - dx[idx]) <= 1e-5 * (1 + abs(g))
    for idx in [(0, 0), (1, 7), (1, n - 1)]:
        assert abs(fd(B, idx, lambda a: L(x, a, G, S)) - dB[idx]) <= 1e-5 * (1 + abs(dB[idx]))
        assert abs(fd(G, idx, lambda a: L(x, B, a, S)) - dG[idx]) <= 1e-5 * (1 + abs(dG[idx]))
        assert abs(fd(S, idx, lambda a: L(x, B, G, a)) - dS[idx]) <= 1e-4 * (1 + abs(dS[idx]))


def test_adjoint_torch_gradcheck(orc):
    torch = pytest.importorskip("torch")
    n, E, d = 8, 2, 7
    p = orc.params(21, n, E, 0.7)
    perm = p["perm"]

    class F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, B, G, S):
            ctx.save_for_backward(x, B, G, S)
            z = orc.project(x.numpy(), n, E, B.numpy(), perm, G.numpy(), S.numpy())
            return torch.from_numpy(orc.features(z, n, E))

        @staticmethod
        def backward(ctx, g):
            x, B, G, S = ctx.saved_tensors
            dx, dB, dG, dS = orc.backward(x.numpy(), g.contiguous().numpy(), n, E, B.numpy(), perm,
                                          G.numpy(), S.numpy())
            return tuple(torch.from_numpy(a) for a in (dx, dB, dG, dS))

    gen = torch.Generator().manual_seed(0)
    x = torch.randn(3, d, dtype=torch.float64, generator=gen, requires_grad=True)
    B = torch.from_numpy(p["B"].astype(np.float64)).requires_grad_()
    G = torch.from_numpy(p["G"].astype(np.float64)).requires_grad_()
    S = torch.from_numpy(p["S64"]).requires_grad_()
    assert torch.autograd.gradcheck(F.apply, (x, B, G, S), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_generator_deterministic_and_seed_dependent(orc):
    a = orc.params(1, 64, 2, 1.0)
    b = orc.params(1, 64, 2, 1.0)
    c = orc.params(2, 64, 2, 1.0)
    for k in ("B", "perm", "G", "S64"):
        np.testing.assert_array_equal(a[k], b[k])
    assert not np.array_equal(a["G"], c["G"])
    assert not np.array_equal(a["G"][0], a["G"][1])  # expansions drawn independently
