"""FP64 CPU oracle of the Fastfood feature map (McKernel, sections "McKernel"
and "Fast Walsh Hadamard").

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product package never
imports it.  It wraps ``oracle.c`` (plain C, built with ``-ffp-contract=off``)
through ctypes and numpy; nothing here touches a GPU.

Functions (all FP64 unless the generator's definition fixes the precision):
  hash4, murmur3          -- MurmurHash3_x86_32 (the hash named for B, Pi, G)
  ln32, sincos2pi32       -- FP32 elementary functions of the G generator
  ln64, cos2pi64          -- FP64 elementary functions of the S generator
  boxmuller32, normal64, chi
  params(seed, n, E, sigma, matern_t) -- B, perm, G, S64, S32 (RBF, or RBF-Matern)
  ball_sample, matern                  -- the RBF-Matern calibration draws
  fwht(v)                              -- H v by the divide-and-conquer recursion
  project(x, n, E, B, perm, G, S)      -- z = S H G Pi H B xhat per expansion
  features(z, n, E)                    -- c [cos z, sin z]
  forward(x, E, seed, sigma)           -- phi in FP64 from the generated parameters
  backward(x, dphi, n, E, B, perm, G, S) -- dx, dB, dG, dS
  softmax_xent(logits, labels)         -- mean cross-entropy and d/dlogits
  train_step(x, labels, W, b, B, perm, G, S) -- loss and every gradient of the
                                          softmax(W phi + b) classifier
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u32, i64, f32, f64 = ctypes.c_uint32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    vp = ctypes.c_void_p
    lib.orc_murmur3_x86_32.restype = u32
    lib.orc_murmur3_x86_32.argtypes = [ctypes.c_char_p, i64, u32]
    lib.orc_hash4.restype = u32
    lib.orc_hash4.argtypes = [u32, u32, u32, u32, u32]
    lib.orc_ln32.restype = f32
    lib.orc_ln32.argtypes = [f32]
    lib.orc_sincos2pi32.restype = None
    lib.orc_sincos2pi32.argtypes = [u32, ctypes.POINTER(f32), ctypes.POINTER(f32)]
    lib.orc_boxmuller32.restype = None
    lib.orc_boxmuller32.argtypes = [u32, u32, ctypes.POINTER(f32), ctypes.POINTER(f32)]
    lib.orc_boxmuller32_many.restype = None
    lib.orc_boxmuller32_many.argtypes = [vp, vp, i64, vp, vp]
    lib.orc_ln64.restype = f64
    lib.orc_ln64.argtypes = [f64]
    lib.orc_cos2pi64.restype = f64
    lib.orc_cos2pi64.argtypes = [u32]
    lib.orc_normal64.restype = f64
    lib.orc_normal64.argtypes = [u32, u32]
    lib.orc_chi.restype = f64
    lib.orc_chi.argtypes = [u32, i64, i64, i64]
    lib.orc_padded_dim.restype = i64
    lib.orc_padded_dim.argtypes = [i64]
    lib.orc_params.restype = ctypes.c_int
    lib.orc_params.argtypes = [u32, i64, i64, f64, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_params_c.restype = ctypes.c_int
    lib.orc_params_c.argtypes = [u32, i64, i64, f64, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_ball_sample.restype = None
    lib.orc_ball_sample.argtypes = [u32, i64, u32, i64, vp]
    lib.orc_matern.restype = f64
    lib.orc_matern.argtypes = [u32, i64, i64, i64, i64]
    lib.orc_fwht.restype = ctypes.c_int
    lib.orc_fwht.argtypes = [vp, i64, i64]
    lib.orc_project.restype = ctypes.c_int
    lib.orc_project.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp, vp, vp]
    lib.orc_features.restype = ctypes.c_int
    lib.orc_features.argtypes = [vp, i64, i64, i64, vp]
    lib.orc_backward.restype = ctypes.c_int
    lib.orc_backward.argtypes = [vp, vp, i64, i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- hash
def murmur3(key: bytes, seed: int) -> int:
    return int(_load().orc_murmur3_x86_32(key, len(key), seed & 0xFFFFFFFF))


def hash4(seed: int, w0: int, w1: int, w2: int, w3: int) -> int:
    return int(_load().orc_hash4(seed & 0xFFFFFFFF, w0, w1, w2, w3))


# ---------------------------------------------------------------- generator pieces
def ln32(u: float) -> np.float32:
    return np.float32(_load().orc_ln32(float(u)))


def sincos2pi32(k24: int):
    c, s = ctypes.c_float(), ctypes.c_float()
    _load().orc_sincos2pi32(k24, ctypes.byref(c), ctypes.byref(s))
    return np.float32(c.value), np.float32(s.value)


def boxmuller32(a: int, b: int):
    g0, g1 = ctypes.c_float(), ctypes.c_float()
    _load().orc_boxmuller32(a, b, ctypes.byref(g0), ctypes.byref(g1))
    return np.float32(g0.value), np.float32(g1.value)


def boxmuller32_many(a, b):
    """Vectorised boxmuller32 over uint32 arrays a, b."""
    a = _c(a, np.uint32)
    b = _c(b, np.uint32)
    g0 = np.empty(a.shape, np.float32)
    g1 = np.empty(a.shape, np.float32)
    _load().orc_boxmuller32_many(_ptr(a), _ptr(b), a.size, _ptr(g0), _ptr(g1))
    return g0, g1


def ln64(v: float) -> float:
    return float(_load().orc_ln64(float(v)))


def cos2pi64(h: int) -> float:
    return float(_load().orc_cos2pi64(h))


def normal64(ha: int, hb: int) -> float:
    return float(_load().orc_normal64(ha, hb))


def chi(seed: int, e: int, j: int, n: int) -> float:
    return float(_load().orc_chi(seed & 0xFFFFFFFF, e, j, n))


def padded_dim(d: int) -> int:
    return int(_load().orc_padded_dim(d))


# ---------------------------------------------------------------- parameters
def ball_sample(seed: int, e: int, w: int, n: int) -> np.ndarray:
    """One sample uniform in the unit n-ball (the RBF-Matern building block)."""
    z = np.empty(n, np.float64)
    _load().orc_ball_sample(seed & 0xFFFFFFFF, e, w & 0xFFFFFFFF, n, _ptr(z))
    return z


def matern(seed: int, e: int, j: int, n: int, t: int) -> float:
    """RBF-Matern radius: the norm of the sum of t unit-ball samples."""
    return _load().orc_matern(seed & 0xFFFFFFFF, e, j, n, t)


def params(seed: int, n: int, E: int, sigma: float, with_aux: bool = False, matern_t: int = 0):
    """B, perm, G (E x n; float32, int32, float32), S64 (float64) and S32
    (float32).  With ``with_aux`` also the calibration radii s_j (chi(n), or
    the RBF-Matern radii when matern_t > 0) and ||G_e||^2."""
    B = np.empty((E, n), np.float32)
    P = np.empty((E, n), np.int32)
    G = np.empty((E, n), np.float32)
    S64 = np.empty((E, n), np.float64)
    S32 = np.empty((E, n), np.float32)
    chi_ = np.empty((E, n), np.float64) if with_aux else None
    nrm = np.empty((E,), np.float64) if with_aux else None
    rc = _load().orc_params_c(seed & 0xFFFFFFFF, n, E, float(sigma), int(matern_t), _ptr(B), _ptr(P),
                              _ptr(G), _ptr(S64), _ptr(S32), _ptr(chi_), _ptr(nrm))
    if rc != 0:
        raise ValueError("orc_params rejected (n=%d, E=%d, sigma=%r)" % (n, E, sigma))
    out = {"B": B, "perm": P, "G": G, "S64": S64, "S32": S32}
    if with_aux:
        out["chi"] = chi_
        out["norm2"] = nrm
    return out


# ---------------------------------------------------------------- transform
def fwht(v) -> np.ndarray:
    """H v along the last axis (unnormalised Sylvester order), FP64."""
    a = np.array(v, dtype=np.float64, copy=True)
    n = a.shape[-1]
    flat = np.ascontiguousarray(a.reshape(-1, n))
    if _load().orc_fwht(_ptr(flat), flat.shape[0], n) != 0:
        raise ValueError("n must be a power of two")
    return flat.reshape(a.shape)


def project(x, n: int, E: int, B, perm, G, S) -> np.ndarray:
    """z (batch x E n) for explicit diagonals (S includes every scale)."""
    x = _c(np.atleast_2d(x), np.float64)
    batch, d = x.shape
    B, G, S = (_c(a, np.float64).reshape(E, n) for a in (B, G, S))
    perm = _c(perm, np.int32).reshape(E, n)
    z = np.empty((batch, E * n), np.float64)
    if _load().orc_project(_ptr(x), batch, d, n, E, _ptr(B), _ptr(perm), _ptr(G),
                           _ptr(S), _ptr(z)) != 0:
        raise ValueError("orc_project rejected its arguments")
    return z


def features(z, n: int, E: int) -> np.ndarray:
    z = _c(np.atleast_2d(z), np.float64)
    phi = np.empty((z.shape[0], 2 * n * E), np.float64)
    if _load().orc_features(_ptr(z), z.shape[0], n, E, _ptr(phi)) != 0:
        raise ValueError("orc_features rejected its arguments")
    return phi


def forward(x, E: int, seed: int, sigma: float, p=None, matern_t: int = 0):
    """phi (batch x 2nE, FP64) with the generated parameters (FP32 G promoted,
    FP64 S).  Returns (phi, z, params)."""
    x = np.atleast_2d(x)
    n = padded_dim(x.shape[1])
    if p is None:
        p = params(seed, n, E, sigma, matern_t=matern_t)
    z = project(x, n, E, p["B"], p["perm"], p["G"], p["S64"])
    return features(z, n, E), z, p


def backward(x, dphi, n: int, E: int, B, perm, G, S):
    """(dx, dB, dG, dS) of <dphi, phi(x)> for explicit diagonals, FP64."""
    x = _c(np.atleast_2d(x), np.float64)
    batch, d = x.shape
    dphi = _c(dphi, np.float64).reshape(batch, 2 * n * E)
    B, G, S = (_c(a, np.float64).reshape(E, n) for a in (B, G, S))
    perm = _c(perm, np.int32).reshape(E, n)
    dx = np.empty((batch, d), np.float64)
    dB = np.empty((E, n), np.float64)
    dG = np.empty((E, n), np.float64)
    dS = np.empty((E, n), np.float64)
    if _load().orc_backward(_ptr(x), _ptr(dphi), batch, d, n, E, _ptr(B), _ptr(perm),
                            _ptr(G), _ptr(S), _ptr(dx), _ptr(dB), _ptr(dG), _ptr(dS)) != 0:
        raise ValueError("orc_backward rejected its arguments")
    return dx, dB, dG, dS


# ---------------------------------------------------------------- training step
def softmax_xent(logits, labels):
    """Mean cross-entropy of softmax(logits) against integer labels, and its
    gradient with respect to the logits, FP64."""
    lg = np.asarray(logits, np.float64)
    y = np.asarray(labels, np.int64)
    m = lg.max(axis=1, keepdims=True)
    ex = np.exp(lg - m)
    s = ex.sum(axis=1, keepdims=True)
    logp = lg - m - np.log(s)
    batch = lg.shape[0]
    loss = -logp[np.arange(batch), y].mean()
    dlog = ex / s
    dlog[np.arange(batch), y] -= 1.0
    return loss, dlog / batch


def train_step(x, labels, W, b, B, perm, G, S):
    """One softmax(W phi(x) + b) cross-entropy step with explicit diagonals
    (section "Empirical Analysis and Experiments": the classifier on the
    McKernel features; section "Large-scale Machine Learning": minimised by
    SGD).  Returns the mean loss and the gradients with respect to W, b, x,
    B, G, S, all FP64."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    W = np.asarray(W, np.float64)
    b = np.asarray(b, np.float64)
    E, n = np.asarray(B).reshape(-1, np.asarray(B).shape[-1]).shape
    z = project(x, n, E, B, perm, G, S)
    phi = features(z, n, E)
    logits = phi @ W.T + b
    loss, dlog = softmax_xent(logits, labels)
    dW = dlog.T @ phi
    db = dlog.sum(axis=0)
    dphi = dlog @ W
    dx, dB, dG, dS = backward(x, dphi, n, E, B, perm, G, S)
    return {"loss": loss, "dW": dW, "db": db, "dx": dx, "dB": dB, "dG": dG, "dS": dS, "logits": logits}
