"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers; it holds none of the feature map's
arithmetic.  The inputs stand in for MNIST / FASHION-MNIST (28 x 28 = 784
values per image in [0, 1], used in the paper's experiments section) which
are not available here: same shape, same value range, synthetic values.

Recipes (numpy ``default_rng``; float32 unless stated):
  mnist_uniform(batch, seed=0)  -- rng.random((batch, 784))            [dense images]
  mnist_sparse(batch, seed=0)   -- v = rng.random((batch, 784)); keep = rng.random(...) >= 0.8;
                                   x = where(keep, v, 0)               [80 % zero pixels]
  normal(batch, d, seed)        -- rng.standard_normal((batch, d))
  grad_features(batch, width, seed=1) -- rng.standard_normal((batch, width)), the
                                   cotangent fed to the backward pass
  ragged_instances(count, seed=0) -- list of (n, batch, E) with n = 2^U{8..16},
                                   batch U{16..4096}, E U{1..16}
"""
from __future__ import annotations

import numpy as np

MNIST_D = 784
FASTFOOD_SEED = 1398239763  # the seed used in the paper's experiments


def mnist_uniform(batch: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((batch, MNIST_D), dtype=np.float32)


def mnist_sparse(batch: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.random((batch, MNIST_D), dtype=np.float32)
    keep = rng.random((batch, MNIST_D)) >= 0.8
    return np.where(keep, v, np.float32(0)).astype(np.float32)


def normal(batch: int, d: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, d), dtype=np.float32)


def grad_features(batch: int, width: int, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, width), dtype=np.float32)


def ragged_instances(count: int = 32, seed: int = 0):
    rng = np.random.default_rng(seed)
    ms, bs, es = rng.integers(8, 17, count), rng.integers(16, 4097, count), rng.integers(1, 17, count)
    return [(1 << int(m), int(b), int(e)) for m, b, e in zip(ms, bs, es)]
