"""CPU pins of the oracle's RBF-Matern calibration (section "Customizing
McKernel": C_kk is the Euclidean norm of the sum of t i.i.d. samples drawn
uniformly from the unit n-ball, each drawn as U^(1/n) X / ||X||).

Each pin is fixed by the mathematics, not by the oracle's own formulas:
the radius law P(||Z|| <= r) = r^n of a uniform ball sample, E||Z||^2 =
n/(n+2), zero mean, the t = 1 case reducing to U^(1/n) (against libm's
pow), E C^2 = t n/(n+2) for a sum of independent zero-mean samples, the
row-norm identity of the resulting Z (row norms C_j / sigma exactly), and
the kernel E_seed[phi(x).phi(y)] against an independent Monte Carlo of the
same spectral law built from numpy's own random numbers."""
import numpy as np
import pytest
import scipy.linalg
import scipy.stats


def test_single_sample_radius_is_u_to_the_one_over_n(orc):
    seed = 1398239763
    for n in (2, 8, 64, 1024):
        for j in range(5):
            hu = orc.hash4(seed, 5, 3, j, 0)  # tag 5: the sample's uniform
            u = (hu + 1) * 2.0**-32
            c = orc.matern(seed, 3, j, n, 1)
            assert c == pytest.approx(u ** (1.0 / n), rel=4e-16 * np.log2(n) + 1e-15)


@pytest.mark.parametrize("n", [4, 16])
def test_ball_sample_radius_law(orc, n):
    r = np.array([np.linalg.norm(orc.ball_sample(7, 1, w, n)) for w in range(3000)])
    assert r.max() <= 1.0
    # P(R <= r) = r^n
    assert scipy.stats.kstest(r, lambda v: np.clip(v, 0, 1) ** n).pvalue > 1e-3


def test_ball_sample_moments(orc):
    n, m = 8, 4000
    Z = np.array([orc.ball_sample(11, 0, w, n) for w in range(m)])
    sq = (Z**2).sum(axis=1)
    # E||Z||^2 = n / (n + 2); Var||Z||^2 = n/(n+4) - (n/(n+2))^2
    var = n / (n + 4) - (n / (n + 2)) ** 2
    assert abs(sq.mean() - n / (n + 2)) <= 4 * np.sqrt(var / m)
    # zero mean, isotropic: each coordinate has variance 1/(n+2)
    se = np.sqrt(1.0 / (n + 2) / m)
    assert np.all(np.abs(Z.mean(axis=0)) <= 4.5 * se)


def test_sum_of_samples_second_moment(orc):
    n, t, E = 16, 40, 8
    p = orc.params(5, n, E, 1.0, with_aux=True, matern_t=t)
    c2 = (p["chi"] ** 2).ravel()
    # independent zero-mean samples: E C^2 = t E||Z||^2 = t n / (n + 2)
    expect = t * n / (n + 2)
    assert abs(c2.mean() - expect) <= 4 * c2.std() / np.sqrt(c2.size)


@pytest.mark.parametrize("n,sigma", [(16, 1.0), (64, 0.7)])
def test_matern_row_norm_identity(orc, n, sigma):
    # Same derivation as for the RBF scaling: the rows of Z have norm C_j / sigma.
    E, t = 2, 40
    p = orc.params(2024, n, E, sigma, with_aux=True, matern_t=t)
    Z = orc.project(np.eye(n), n, E, p["B"], p["perm"], p["G"], p["S64"])
    for e in range(E):
        Ze = Z[:, e * n:(e + 1) * n].T
        np.testing.assert_allclose(np.linalg.norm(Ze, axis=1), p["chi"][e] / sigma, rtol=1e-12)


def test_matern_kernel_against_independent_monte_carlo(orc):
    # E_seed[phi(x).phi(y)] = E[cos(w.(x - y))] with w = (C / sigma) u, u a
    # uniform direction and C the norm of a sum of t unit-ball samples.  The
    # reference draws C and u from numpy's generator (independent of the hash).
    n, E, t, sigma = 16, 4, 40, 1.0
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, n)) * 0.15
    y = x + rng.standard_normal((1, n)) * 0.15
    vals = []
    for seed in range(120):
        phi, _, _ = orc.forward(np.vstack([x, y]), E, seed, sigma, matern_t=t)
        vals.append(float(phi[0] @ phi[1]))
    vals = np.array(vals)
    m = 200000
    X = rng.standard_normal((m, t, n))
    U = rng.random((m, t, 1))
    Zs = (U ** (1.0 / n)) * X / np.linalg.norm(X, axis=2, keepdims=True)
    C = np.linalg.norm(Zs.sum(axis=1), axis=1)
    u = rng.standard_normal((m, n))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    k_ref = np.cos((C / sigma) * (u @ (x - y).ravel())).mean()
    se = np.sqrt(vals.var() / len(vals) + 1.0 / m)
    assert abs(vals.mean() - k_ref) <= 4 * se
    # and it is not the RBF kernel exp(-|x-y|^2 / 2 sigma^2) (different spectral law)
    k_rbf = np.exp(-np.sum((x - y) ** 2) / (2 * sigma**2))
    assert abs(k_ref - k_rbf) > 8 * se
