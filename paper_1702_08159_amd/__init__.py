"""MI355X-native Fastfood feature map (McKernel, arXiv 1702.08159).

Python binding of libmckernel.so: argument marshalling only.  Every step of
the computation runs in the library's HIP kernels; tensors must be float32
CUDA (ROCm) tensors on the current device, and work is enqueued on torch's
current stream.

    phi = fastfood(x, E=16, seed=1398239763, sigma=2.0)   # autograd w.r.t. x
    phi = forward(x, E, seed, sigma, out_dtype=torch.bfloat16)  # 16-bit storage
    phi = forward(x, E, seed, sigma, matern_t=40)         # RBF-Matern calibration
    phis = forward_batched([(x1, E1, s1, g1), (x2, E2, s2, g2)])  # uneven maps
    z = project(x, E, seed, sigma)                        # Z xhat, no trig
    p = params(seed, n, E, sigma)                         # generated B, perm, G, S
    y = fwht(v)                                           # H v along the last axis (n <= 2^24)
    phi = FastfoodExplicit.apply(x, B, perm, G, S)        # learnable diagonals
    out = train_step(x, labels, W, b, B, perm, G, S, lr)  # softmax(W phi + b) SGD step
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MCK_CALIB_RBF, MckError


def calibration(matern_t: int = 0) -> int:
    """C-ABI calibration code: RBF (t = 0) or RBF-Matern with t unit-ball samples."""
    if matern_t == 0:
        return MCK_CALIB_RBF
    if not 1 <= matern_t <= 255:
        raise ValueError("matern_t must be in 1..255")
    return 1 if matern_t == 40 else 0x100 + matern_t

PAPER_SEED = 1398239763
MAX_N = 32768

__all__ = ["padded_dim", "fwht", "fwht_", "params", "forward", "project", "backward", "forward_p",
           "backward_p", "fastfood", "FastfoodFunction", "FastfoodExplicit", "gen_boxmuller", "shutdown",
           "MckError", "PAPER_SEED", "MAX_N", "forward_batched", "autotune_batched", "forward_tuning",
           "set_forward_tuning", "BatchedGraph", "forward_scaled", "backward_launch_shape"]


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t: torch.Tensor, name: str, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def padded_dim(d: int) -> int:
    return int(_lib.lib().mck_padded_dim(d))


def fwht_(v: torch.Tensor) -> torch.Tensor:
    """In-place H v along the last axis (unnormalised, natural order)."""
    _check(v, "v")
    n = v.shape[-1]
    with torch.cuda.device(v.device):
        _lib.call("mck_fwht", _ptr(v), v.numel() // max(n, 1), n, _stream(v))
    return v


def fwht(v: torch.Tensor) -> torch.Tensor:
    return fwht_(v.contiguous().clone())


def params(seed: int, n: int, E: int, sigma: float, device=None, matern_t: int = 0):
    """Generated B, perm, G, S (FP32) and S64 (FP64) of a seed-mode plan (E x n)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = {
        "B": torch.empty((E, n), dtype=torch.float32, device=dev),
        "perm": torch.empty((E, n), dtype=torch.int32, device=dev),
        "G": torch.empty((E, n), dtype=torch.float32, device=dev),
        "S": torch.empty((E, n), dtype=torch.float32, device=dev),
        "S64": torch.empty((E, n), dtype=torch.float64, device=dev),
    }
    with torch.cuda.device(dev):
        _lib.call("mck_fastfood_params", seed & 0xFFFFFFFF, n, E, float(sigma), calibration(matern_t), _ptr(out["B"]),
                  _ptr(out["perm"]), _ptr(out["G"]), _ptr(out["S"]), _ptr(out["S64"]),
                  _stream(out["B"]))
    return out


def _rows(x: torch.Tensor):
    if x.dim() != 2:
        raise ValueError("x must be 2-D (batch x d)")
    return x.shape[0], x.shape[1]


_DTYPES = {torch.float32: 0, torch.bfloat16: 1, torch.float16: 2}


def forward(x: torch.Tensor, E: int, seed: int = PAPER_SEED, sigma: float = 1.0, out=None,
            out_dtype=None, matern_t: int = 0) -> torch.Tensor:
    """phi(x): batch x 2nE features [cos blocks, sin blocks].  x may be
    float32, bfloat16 or float16; phi is float32 unless out_dtype (or out)
    says bfloat16 / float16 (16-bit storage, FP32 arithmetic)."""
    if x.dtype != torch.float32 or (out_dtype not in (None, torch.float32)) or (
            out is not None and out.dtype != torch.float32):
        return _forward_t(x, E, seed, sigma, out, out_dtype, matern_t)
    _check(x, "x")
    batch, d = _rows(x)
    n = padded_dim(d)
    if out is None:
        out = torch.empty((batch, 2 * n * E), dtype=torch.float32, device=x.device)
    _check(out, "out")
    with torch.cuda.device(x.device):
        _lib.call("mck_fastfood_forward", _ptr(x), batch, d, E, seed & 0xFFFFFFFF, float(sigma), calibration(matern_t),
                  _ptr(out), _stream(x))
    return out


def _forward_t(x, E, seed, sigma, out, out_dtype, matern_t=0):
    if x.dtype not in _DTYPES:
        raise TypeError("x must be float32, bfloat16 or float16")
    _check(x, "x", x.dtype)
    batch, d = _rows(x)
    n = padded_dim(d)
    if out is None:
        out = torch.empty((batch, 2 * n * E), dtype=out_dtype or x.dtype, device=x.device)
    if out.dtype not in _DTYPES:
        raise TypeError("phi must be float32, bfloat16 or float16")
    _check(out, "out", out.dtype)
    with torch.cuda.device(x.device):
        _lib.call("mck_fastfood_forward_t", _ptr(x), _DTYPES[x.dtype], batch, d, E, seed & 0xFFFFFFFF,
                  float(sigma), calibration(matern_t), _ptr(out), _DTYPES[out.dtype], _stream(x))
    return out


def forward_scaled(x: torch.Tensor, E: int, seed: int = PAPER_SEED, sigma: float = 1.0, x_exp=None,
                   out_dtype=None, matern_t: int = 0):
    """phi with per-row power-of-2 scaling of its storage: x (float32,
    bfloat16 or float16) holds rows x_true[r] / 2^x_exp[r] (x_exp: int8 per
    row, or None); returns (phi_stored, phi_exp) with phi = phi_stored *
    2^-phi_exp[r] per row."""
    if x.dtype not in _DTYPES:
        raise TypeError("x must be float32, bfloat16 or float16")
    _check(x, "x", x.dtype)
    batch, d = _rows(x)
    n = padded_dim(d)
    if x_exp is not None:
        _check(x_exp, "x_exp", torch.int8)
        if x_exp.shape != (batch,):
            raise ValueError("x_exp must hold one exponent per row")
    out = torch.empty((batch, 2 * n * E), dtype=out_dtype or x.dtype, device=x.device)
    phi_exp = torch.empty((batch,), dtype=torch.int8, device=x.device)
    with torch.cuda.device(x.device):
        _lib.call("mck_fastfood_forward_scaled", _ptr(x), _DTYPES[x.dtype], _ptr(x_exp), batch, d, E,
                  seed & 0xFFFFFFFF, float(sigma), calibration(matern_t), _ptr(out), _DTYPES[out.dtype],
                  _ptr(phi_exp), _stream(x))
    return out, phi_exp


def _instances(maps, outs):
    """mck_instance array, the phi list and the device of a batched call.
    Fields are written into one preallocated ctypes array (no per-map ctypes
    temporaries), so marshalling many small maps stays cheap."""
    count = len(maps)
    arr = (_lib.Instance * count)()
    res = []
    dev = maps[0][0].device if count else None
    f32 = torch.float32
    for k in range(count):
        m = maps[k]
        x, E, seed, sigma = m[0], m[1], m[2], m[3]
        mt = m[4] if len(m) > 4 else 0
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != f32 or not x.is_contiguous():
            _check(x, "x")  # raises with the reason
        if x.device != dev:
            raise ValueError("all maps must be on one device")
        if x.dim() != 2:
            raise ValueError("x must be 2-D (batch x d)")
        batch, d = x.shape
        if not 1 <= d <= 1 << 24:
            raise ValueError("d out of range")
        n = max(2, 1 << (d - 1).bit_length())
        if outs is not None:
            phi = outs[k]
            if not isinstance(phi, torch.Tensor) or not phi.is_cuda or phi.dtype != f32 or not phi.is_contiguous():
                _check(phi, "phi")
            if phi.shape != (batch, 2 * n * E):
                raise ValueError("phi must be batch x 2nE")
        else:
            phi = torch.empty((batch, 2 * n * E), dtype=f32, device=dev)
        q = arr[k]
        q.x = x.data_ptr()
        q.batch = batch
        q.d = d
        q.E = E
        q.seed = seed & 0xFFFFFFFF
        q.sigma = sigma
        q.calib = MCK_CALIB_RBF if mt == 0 else calibration(mt)
        q.phi = phi.data_ptr()
        res.append(phi)
    return arr, res, dev


def forward_batched(maps, outs=None):
    """Several independent feature maps in one call: `maps` is a list of
    (x, E, seed, sigma) or (x, E, seed, sigma, matern_t); returns the list of
    phi (FP32).  Maps of the same n share one grouped launch."""
    maps = list(maps)
    if not maps:
        return []
    arr, res, dev = _instances(maps, outs)
    with torch.cuda.device(dev):
        _lib.call("mck_fastfood_forward_batched", ctypes.cast(arr, ctypes.c_void_p), len(maps),
                  _stream(maps[0][0]))
    return res


class BatchedGraph:
    """A batched call recorded once into a HIP graph by the library
    (mck_batched_graph_create) and replayed with launch(): `maps` as for
    forward_batched; `phis` are the output tensors every launch rewrites.
    The tensors of `maps` and `phis` must stay alive while the object does."""

    def __init__(self, maps, outs=None):
        maps = list(maps)
        if not maps:
            raise ValueError("no maps")
        arr, self.phis, self.device = _instances(maps, outs)
        self._keep = ([m[0] for m in maps], self.phis)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.call("mck_batched_graph_create", ctypes.cast(arr, ctypes.c_void_p), len(maps),
                      _stream(maps[0][0]), ctypes.byref(self._h))

    def launch(self):
        with torch.cuda.device(self.device):
            _lib.call("mck_batched_graph_launch", self._h, _stream(self.phis[0]))
        return self.phis

    def close(self):
        if self._h:
            _lib.lib().mck_batched_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_batched(maps, outs=None, reps: int = 3):
    """Times the launch choices for every n <= 2^15 among `maps` (as for
    forward_batched) and keeps the fastest per n; returns {n: (split, waves)}.
    Synchronizes the current stream; writes phi of the timed maps."""
    maps = list(maps)
    if not maps:
        return {}
    arr, res, dev = _instances(maps, outs)
    with torch.cuda.device(dev):
        _lib.call("mck_autotune_forward_batched", ctypes.cast(arr, ctypes.c_void_p), len(maps), int(reps),
                  _stream(maps[0][0]))
        ns = sorted({r.shape[1] // (2 * m[1]) for r, m in zip(res, maps)})
        return {n: forward_tuning(n) for n in ns if n <= MAX_N}


def forward_tuning(n: int):
    """(split, waves) the forward of length n launches with on the current device."""
    t = _lib.ForwardTuning()
    _lib.call("mck_forward_tuning_get", int(n), ctypes.byref(t))
    return (t.split, t.waves)


def set_forward_tuning(n: int, split=None, waves=None):
    """Sets the launch choice for n; split=None and waves=None restore the default."""
    if split is None and waves is None:
        _lib.call("mck_forward_tuning_set", int(n), None)
        return
    cur = forward_tuning(n)
    t = _lib.ForwardTuning(int(split if split is not None else cur[0]), int(waves if waves is not None else cur[1]))
    _lib.call("mck_forward_tuning_set", int(n), ctypes.byref(t))


def project(x: torch.Tensor, E: int, seed: int = PAPER_SEED, sigma: float = 1.0, matern_t: int = 0) -> torch.Tensor:
    """z = Z xhat: batch x nE (expansion-major)."""
    _check(x, "x")
    batch, d = _rows(x)
    n = padded_dim(d)
    out = torch.empty((batch, n * E), dtype=torch.float32, device=x.device)
    with torch.cuda.device(x.device):
        _lib.call("mck_fastfood_project", _ptr(x), batch, d, E, seed & 0xFFFFFFFF, float(sigma), calibration(matern_t),
                  _ptr(out), _stream(x))
    return out


def backward(x: torch.Tensor, dphi: torch.Tensor, E: int, seed: int = PAPER_SEED, sigma: float = 1.0,
             need_dx: bool = True, need_params: bool = False, out=None, matern_t: int = 0):
    """(dx, dB, dG, dS) of <dphi, phi(x)>; entries not requested are None.
    `out` may pass preallocated (dx, dB, dG, dS) (None entries are skipped)."""
    _check(x, "x")
    _check(dphi, "dphi")
    batch, d = _rows(x)
    n = padded_dim(d)
    if dphi.shape != (batch, 2 * n * E):
        raise ValueError("dphi must be batch x 2nE")
    if out is not None:
        dx, dB, dG, dS = out
        if dx is not None:
            _check(dx, "dx")
            if dx.shape != x.shape:
                raise ValueError("dx must have the shape of x")
        for t, nm in ((dB, "dB"), (dG, "dG"), (dS, "dS")):
            if t is not None:
                _check(t, nm)
                if t.numel() != E * n:
                    raise ValueError(nm + " must hold E x n values")
    else:
        dx = torch.empty_like(x) if need_dx else None
        dB = dG = dS = None
        if need_params:
            dB, dG, dS = (torch.empty((E, n), dtype=torch.float32, device=x.device) for _ in range(3))
    with torch.cuda.device(x.device):
        _lib.call("mck_fastfood_backward", _ptr(x), _ptr(dphi), batch, d, E, seed & 0xFFFFFFFF, float(sigma),
                  calibration(matern_t), _ptr(dx), _ptr(dB), _ptr(dG), _ptr(dS), _stream(x))
    return dx, dB, dG, dS


def forward_p(x, B, perm, G, S) -> torch.Tensor:
    """phi(x) for explicit diagonals B, G, S (E x n float32) and perm (E x n int32)."""
    _check(x, "x")
    for t, nm in ((B, "B"), (G, "G"), (S, "S")):
        _check(t, nm)
    _check(perm, "perm", torch.int32)
    batch, d = _rows(x)
    E, n = B.shape
    out = torch.empty((batch, 2 * n * E), dtype=torch.float32, device=x.device)
    with torch.cuda.device(x.device):
        _lib.call("mck_fastfood_forward_p", _ptr(x), batch, d, n, E, _ptr(B), _ptr(perm), _ptr(G), _ptr(S),
                  _ptr(out), _stream(x))
    return out


def backward_launch_shape(batch: int, d: int, E: int) -> dict:
    """Launch shape of the adjoint for (batch, d, E): rows_per_pass, passes,
    esplit, rowblocks (a host query; nothing runs on the GPU)."""
    sh = _lib.BackwardShape()
    _lib.call("mck_backward_launch_shape", batch, d, E, ctypes.byref(sh))
    return {"rows_per_pass": sh.rows_per_pass, "passes": sh.passes, "esplit": sh.esplit,
            "rowblocks": sh.rowblocks}


def backward_p(x, dphi, B, perm, G, S, need_dx=True, need_params=True, out=None, noalloc=False):
    """dx, dB, dG, dS of <dphi, phi> for explicit diagonals.  out: optional
    (dx, dB, dG, dS) tensors to write (None entries are skipped).  noalloc:
    call mck_fastfood_backward_p_noalloc, whose temporaries live in the
    library's static device scratch (the library allocates nothing)."""
    _check(x, "x")
    _check(dphi, "dphi")
    batch, d = _rows(x)
    E, n = B.shape
    if out is not None:
        dx, dB, dG, dS = out
    else:
        dx = torch.empty_like(x) if need_dx else None
        dB = dG = dS = None
        if need_params:
            dB, dG, dS = (torch.empty((E, n), dtype=torch.float32, device=x.device) for _ in range(3))
    name = "mck_fastfood_backward_p_noalloc" if noalloc else "mck_fastfood_backward_p"
    with torch.cuda.device(x.device):
        _lib.call(name, _ptr(x), _ptr(dphi), batch, d, n, E, _ptr(B), _ptr(perm), _ptr(G),
                  _ptr(S), _ptr(dx), _ptr(dB), _ptr(dG), _ptr(dS), _stream(x))
    return dx, dB, dG, dS


class FastfoodFunction(torch.autograd.Function):
    """phi(x) with seed-generated parameters; backward recomputes the forward."""

    @staticmethod
    def forward(ctx, x, E, seed, sigma):
        ctx.save_for_backward(x)
        ctx.cfg = (E, seed, sigma)
        return forward(x, E, seed, sigma)

    @staticmethod
    def backward(ctx, dphi):
        (x,) = ctx.saved_tensors
        E, seed, sigma = ctx.cfg
        dx = None
        if ctx.needs_input_grad[0]:
            dx, _, _, _ = backward(x, dphi.contiguous(), E, seed, sigma, need_dx=True, need_params=False)
        return dx, None, None, None


class FastfoodExplicit(torch.autograd.Function):
    """phi(x) for learnable diagonals B, G, S (perm fixed)."""

    @staticmethod
    def forward(ctx, x, B, perm, G, S):
        ctx.save_for_backward(x, B, perm, G, S)
        return forward_p(x, B, perm, G, S)

    @staticmethod
    def backward(ctx, dphi):
        x, B, perm, G, S = ctx.saved_tensors
        need_p = any(ctx.needs_input_grad[i] for i in (1, 3, 4))
        dx, dB, dG, dS = backward_p(x, dphi.contiguous(), B, perm, G, S, need_dx=ctx.needs_input_grad[0],
                                    need_params=need_p)
        return dx, dB, None, dG, dS


def fastfood(x: torch.Tensor, E: int, seed: int = PAPER_SEED, sigma: float = 1.0) -> torch.Tensor:
    return FastfoodFunction.apply(x, E, seed, sigma)


def gen_boxmuller(a: torch.Tensor, b: torch.Tensor):
    """Device generator's FP32 Box-Muller pair for hash words a, b (int32 views of uint32)."""
    _check(a, "a", torch.int32)
    _check(b, "b", torch.int32)
    g0 = torch.empty(a.shape, dtype=torch.float32, device=a.device)
    g1 = torch.empty_like(g0)
    with torch.cuda.device(a.device):
        _lib.call("mck_gen_boxmuller", _ptr(a), _ptr(b), a.numel(), _ptr(g0), _ptr(g1), _stream(a))
    return g0, g1


def softmax_xent(logits: torch.Tensor, labels: torch.Tensor):
    """(mean cross-entropy, dlogits, db) of softmax(logits) against int32 labels."""
    _check(logits, "logits")
    _check(labels, "labels", torch.int32)
    batch, C = logits.shape
    if labels.shape != (batch,):
        raise ValueError("labels must have one entry per row")
    loss = torch.empty((), dtype=torch.float32, device=logits.device)
    dlogits = torch.empty_like(logits)
    db = torch.empty((C,), dtype=torch.float32, device=logits.device)
    with torch.cuda.device(logits.device):
        _lib.call("mck_softmax_xent", _ptr(logits), _ptr(labels), batch, C, _ptr(loss), _ptr(dlogits), _ptr(db),
                  _stream(logits))
    return loss, dlogits, db


def axpy_(y: torch.Tensor, x: torch.Tensor, alpha: float) -> torch.Tensor:
    """y += alpha x in place (the SGD update with alpha = -learning rate)."""
    _check(y, "y")
    _check(x, "x")
    if y.numel() != x.numel():
        raise ValueError("y and x must have the same number of elements")
    with torch.cuda.device(y.device):
        _lib.call("mck_axpy", _ptr(y), _ptr(x), y.numel(), float(alpha), _stream(y))
    return y


def head_logits(phi: torch.Tensor, W: torch.Tensor, b=None) -> torch.Tensor:
    """logits = phi W^T + b for C <= 16 classes (phi: batch x F, W: C x F)."""
    _check(phi, "phi")
    _check(W, "W")
    if b is not None:
        _check(b, "b")
    batch, F = phi.shape
    C = W.shape[0]
    if W.shape != (C, F) or (b is not None and b.shape != (C,)):
        raise ValueError("W must be C x F and b of length C")
    logits = torch.empty((batch, C), dtype=torch.float32, device=phi.device)
    with torch.cuda.device(phi.device):
        _lib.call("mck_head_logits", _ptr(phi), _ptr(W), _ptr(b) if b is not None else None, batch, F, C,
                  _ptr(logits), _stream(phi))
    return logits


def head_backward(phi: torch.Tensor, dlogits: torch.Tensor, W: torch.Tensor, need_dphi=True, need_dW=True):
    """(dphi, dW) = (dlogits W, dlogits^T phi); either may be skipped (None)."""
    _check(phi, "phi")
    _check(dlogits, "dlogits")
    _check(W, "W")
    batch, F = phi.shape
    C = W.shape[0]
    if W.shape != (C, F) or dlogits.shape != (batch, C):
        raise ValueError("W must be C x F and dlogits batch x C")
    dphi = torch.empty_like(phi) if need_dphi else None
    dW = torch.empty_like(W) if need_dW else None
    with torch.cuda.device(phi.device):
        _lib.call("mck_head_backward", _ptr(phi), _ptr(dlogits), _ptr(W), batch, F, C,
                  _ptr(dphi) if dphi is not None else None, _ptr(dW) if dW is not None else None, _stream(phi))
    return dphi, dW


def train_step(x, labels, W, b, B, perm, G, S, lr=None, need_dx=False):
    """One step of the classifier softmax(W phi(x) + b) with cross-entropy on
    the features of explicit diagonals B, G, S (perm fixed), as one library
    call: feature map, logits, softmax cross-entropy, the head's products and
    the feature map's adjoint all run in this library's kernels.  Returns the
    loss and the gradients with respect to W, b, B, G, S (and x if need_dx);
    with lr given, applies the SGD update to W, b, B, G, S in place."""
    _check(x, "x")
    _check(labels, "labels", torch.int32)
    for t, nm in ((W, "W"), (b, "b"), (B, "B"), (G, "G"), (S, "S")):
        _check(t, nm)
    _check(perm, "perm", torch.int32)
    batch, d = _rows(x)
    E, n = B.shape
    C = W.shape[0]
    if W.shape != (C, 2 * n * E) or b.shape != (C,) or labels.shape != (batch,):
        raise ValueError("W must be C x 2nE, b of length C and labels of length batch")
    for t in (perm, G, S):
        if t.shape != (E, n):
            raise ValueError("B, perm, G and S must all be E x n")
    dev = x.device
    out = {"loss": torch.empty((), dtype=torch.float32, device=dev),
           "logits": torch.empty((batch, C), dtype=torch.float32, device=dev),
           "dW": torch.empty_like(W), "db": torch.empty_like(b), "dB": torch.empty_like(B),
           "dG": torch.empty_like(G), "dS": torch.empty_like(S),
           "dx": torch.empty((batch, d), dtype=torch.float32, device=dev) if need_dx else None}
    with torch.cuda.device(dev):
        _lib.call("mck_fastfood_train_step", _ptr(x), _ptr(labels), batch, d, n, E, C, _ptr(W), _ptr(b), _ptr(B),
                  _ptr(perm), _ptr(G), _ptr(S), float(lr) if lr is not None else 0.0, _ptr(out["loss"]),
                  _ptr(out["logits"]), _ptr(out["dW"]), _ptr(out["db"]), _ptr(out["dB"]), _ptr(out["dG"]),
                  _ptr(out["dS"]), _ptr(out["dx"]), _stream(x))
    return out


def shutdown() -> None:
    _lib.lib().mck_shutdown()
