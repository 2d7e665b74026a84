"""The C interface loads, exports every declared symbol, and rejects bad
arguments before touching a GPU (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mckernel.h")

pytestmark = pytest.mark.skipif(
    not os.path.exists(os.path.join(ROOT, "paper_1702_08159_amd", "libmckernel.so")),
    reason="libmckernel.so not built (run __graft_entry__.build())")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mck_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1702_08159_amd import _lib

    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    from paper_1702_08159_amd import _lib

    syms = declared_symbols()
    assert len(syms) >= 11
    for s in syms:
        assert hasattr(lib, s), s
        assert s in _lib.SIGNATURES, "binding lacks " + s


def test_padded_dim(lib):
    assert [lib.mck_padded_dim(d) for d in (0, 1, 2, 3, 5, 784, 1024, 1025, 32768, 32769, 1 << 24,
                                            (1 << 24) + 1)] == \
        [0, 2, 2, 4, 8, 1024, 1024, 2048, 32768, 65536, 1 << 24, 0]


def test_status_strings(lib):
    for st in range(5):
        assert lib.mck_status_string(st)
    assert lib.mck_status_string(0) == b"success"


def _st(lib, name, *args):
    return getattr(lib, name)(*args)


def test_validation_without_gpu(lib):
    null = None
    # mck_fwht: n not a power of two, negative batch, n too large, NULL data
    assert _st(lib, "mck_fwht", null, 1, 3, null) == 1
    assert _st(lib, "mck_fwht", null, -1, 4, null) == 1
    assert _st(lib, "mck_fwht", null, 1, 1 << 25, null) == 2
    assert _st(lib, "mck_fwht", ctypes.c_void_p(8), 1, 65536, null) == 1   # unaligned long rows
    assert _st(lib, "mck_fwht", null, 2, 8, null) == 1
    assert b"NULL" in lib.mck_last_error()
    assert _st(lib, "mck_fwht", null, 0, 8, null) == 0       # empty batch
    # forward: d < 1, E < 1, bad sigma, calibration codes, NULL x, too long
    fwd = "mck_fastfood_forward"
    assert _st(lib, fwd, null, 4, 0, 1, 1, 1.0, 0, null, null) == 1
    assert _st(lib, fwd, null, 4, 8, 0, 1, 1.0, 0, null, null) == 1
    for sig in (0.0, -1.0, float("nan"), float("inf")):
        assert _st(lib, fwd, null, 4, 8, 1, 1, sig, 0, null, null) == 1
    # calibrations: unknown codes are invalid; RBF-Matern (1, or 0x100 + t)
    # is accepted up to n = 2048 and unsupported beyond
    for code in (2, 7, 0x100, 0x200, -1):
        assert _st(lib, fwd, null, 4, 8, 1, 1, 1.0, code, null, null) == 1
    assert _st(lib, fwd, null, 4, 3000, 1, 1, 1.0, 1, null, null) == 2
    assert _st(lib, fwd, null, 4, 3000, 1, 1, 1.0, 0x105, null, null) == 2
    assert _st(lib, fwd, null, 4, 8, 1, 1, 1.0, 0, null, null) == 1
    assert _st(lib, fwd, null, 4, (1 << 24) + 1, 1, 1, 1.0, 0, null, null) == 2
    # single-pass calls refuse n > 2^15
    assert _st(lib, "mck_fastfood_project", ctypes.c_void_p(16), 4, 40000, 1, 1, 1.0, 0,
               ctypes.c_void_p(16), null) == 2
    assert _st(lib, "mck_fastfood_backward", ctypes.c_void_p(16), ctypes.c_void_p(16), 4, 40000, 1, 1, 1.0, 0,
               ctypes.c_void_p(16), null, null, null, null) == 2
    assert _st(lib, fwd, null, 0, 8, 2, 1, 1.0, 0, null, null) == 0  # empty batch
    # backward: NULL dphi; nothing requested is a no-op
    bwd = "mck_fastfood_backward"
    assert _st(lib, bwd, null, null, 3, 8, 1, 1, 1.0, 0, ctypes.c_void_p(16), null, null, null, null) == 1
    assert _st(lib, bwd, ctypes.c_void_p(16), ctypes.c_void_p(16), 3, 8, 1, 1, 1.0, 0,
               null, null, null, null, null) == 0
    # explicit forms: n mismatch, NULL parameters
    assert _st(lib, "mck_fastfood_forward_p", null, 1, 8, 16, 1, null, null, null, null, null, null) == 1
    p = ctypes.c_void_p(16)
    assert _st(lib, "mck_fastfood_forward_p", null, 1, 8, 16, 1, p, p, p, p, null, null) == 1
    assert _st(lib, "mck_fastfood_forward_p", null, 1, 8, 8, 1, p, p, p, p, null, null) == 1
    # params: n not a power of two, n = 1, bad sigma, unknown / unsupported calibration
    prm = "mck_fastfood_params"
    assert _st(lib, prm, 1, 12, 1, 1.0, 0, null, null, null, null, null, null) == 1
    assert _st(lib, prm, 1, 1, 1, 1.0, 0, null, null, null, null, null, null) == 1
    assert _st(lib, prm, 1, 8, 1, 0.0, 0, null, null, null, null, null, null) == 1
    assert _st(lib, prm, 1, 8, 1, 1.0, 9, null, null, null, null, null, null) == 1
    assert _st(lib, prm, 1, 4096, 1, 1.0, 1, null, null, null, null, null, null) == 2
    # head products: F not a multiple of 4, too many classes, NULL pointers,
    # nothing requested is a no-op
    p16 = ctypes.c_void_p(16)
    assert _st(lib, "mck_head_logits", p16, p16, null, 2, 6, 10, p16, null) == 1
    assert _st(lib, "mck_head_logits", p16, p16, null, 2, 8, 17, p16, null) == 2
    assert _st(lib, "mck_head_logits", p16, p16, null, 2, 8, 0, p16, null) == 1
    assert _st(lib, "mck_head_logits", null, p16, null, 2, 8, 10, p16, null) == 1
    assert _st(lib, "mck_head_logits", p16, ctypes.c_void_p(20), null, 2, 8, 10, p16, null) == 1
    assert _st(lib, "mck_head_logits", null, null, null, 0, 8, 10, null, null) == 0
    assert _st(lib, "mck_head_backward", p16, null, p16, 2, 8, 10, p16, p16, null) == 1
    assert _st(lib, "mck_head_backward", null, null, null, 2, 8, 10, null, null, null) == 0
    assert _st(lib, "mck_head_backward", p16, p16, null, 2, 8, 10, null, p16, null) == 1  # dW only, W NULL
    assert _st(lib, "mck_head_backward", p16, p16, p16, 2, 8, 10, ctypes.c_void_p(24), null, null) == 1
    # training step: empty batch, too many classes, NULL gradients, bad lr
    ts = "mck_fastfood_train_step"
    args = lambda batch, C, dW, lr: (p16, p16, batch, 8, 8, 1, C, p16, p16, p16, p16, p16, p16, ctypes.c_float(lr),
                                     p16, null, dW, p16, p16, p16, p16, null, null)
    assert _st(lib, ts, *args(0, 10, p16, 0.1)) == 1
    assert _st(lib, ts, *args(4, 17, p16, 0.1)) == 2
    assert _st(lib, ts, *args(4, 10, null, 0.1)) == 1
    assert _st(lib, ts, *args(4, 10, p16, float("nan"))) == 1
    # generator self-check: negative count, NULL pointers
    assert _st(lib, "mck_gen_boxmuller", null, null, -1, null, null, null) == 1
    assert _st(lib, "mck_gen_boxmuller", null, null, 5, null, null, null) == 1
    assert _st(lib, "mck_gen_boxmuller", null, null, 0, null, null, null) == 0


def test_python_binding_refuses_cpu_tensors():
    import torch

    import paper_1702_08159_amd as mk

    with pytest.raises(TypeError):
        mk.forward(torch.zeros(2, 8), 1)
    with pytest.raises(TypeError):
        mk.fwht_(torch.zeros(2, 8))


def test_tuning_and_graph_validation_without_gpu(lib):
    from paper_1702_08159_amd import _lib

    null = None
    t = _lib.ForwardTuning(5, 4096)
    # the tuning table: n must be a power of two in [2, 2^15]; NULL out
    for n in (0, 1, 3, 1000, 65536):
        assert _st(lib, "mck_forward_tuning_get", n, ctypes.byref(t)) == 1
        assert _st(lib, "mck_forward_tuning_set", n, ctypes.byref(t)) == 1
    assert _st(lib, "mck_forward_tuning_get", 1024, null) == 1
    # the autotuner: reps outside [1, 1000]
    assert _st(lib, "mck_autotune_forward_batched", null, 0, 0, null) == 1
    assert _st(lib, "mck_autotune_forward_batched", null, 0, 1001, null) == 1
    # the recorded batched call: NULL out, NULL graph; destroying NULL is a no-op
    assert _st(lib, "mck_batched_graph_create", null, 0, null, null) == 1
    assert _st(lib, "mck_batched_graph_launch", null, null) == 1
    lib.mck_batched_graph_destroy(None)


def test_scaled_forward_validation_without_gpu(lib):
    null = None
    sc = "mck_fastfood_forward_scaled"
    p16 = ctypes.c_void_p(16)
    # unknown storage type, unsupported pair, n too large, NULL x; empty batch is a no-op
    assert _st(lib, sc, p16, 3, null, 2, 8, 1, 1, 1.0, 0, p16, 0, null, null) == 1
    assert _st(lib, sc, p16, 1, null, 2, 8, 1, 1, 1.0, 0, p16, 2, null, null) == 2
    assert _st(lib, sc, p16, 0, p16, 2, (1 << 24) + 1, 1, 1, 1.0, 0, p16, 0, null, null) == 2  # n too large
    assert _st(lib, sc, null, 0, null, 2, 8, 1, 1, 1.0, 0, p16, 0, null, null) == 1
    assert _st(lib, sc, null, 0, null, 0, 8, 1, 1, 1.0, 0, null, 0, null, null) == 0


def test_backward_launch_shape_without_gpu(lib):
    # the host query of the adjoint's launch shape: the metric workload runs
    # four row passes per block over 256 blocks, small batches split the
    # expansions, the LDS caps the passes (4 at d = 784, 3 at d = 1024)
    import paper_1702_08159_amd as mk

    assert mk.backward_launch_shape(8192, 784, 16) == {"rows_per_pass": 8, "passes": 4, "esplit": 1,
                                                       "rowblocks": 256}
    assert mk.backward_launch_shape(1024, 784, 16) == {"rows_per_pass": 8, "passes": 1, "esplit": 2,
                                                       "rowblocks": 128}
    assert mk.backward_launch_shape(8200, 784, 1)["passes"] == 4
    assert mk.backward_launch_shape(8193, 1024, 1)["passes"] == 3
    assert mk.backward_launch_shape(32769, 64, 2) == {"rows_per_pass": 128, "passes": 2, "esplit": 2,
                                                      "rowblocks": 129}
    with pytest.raises(mk.MckError):
        mk.backward_launch_shape(4, 40000, 1)   # beyond the single-pass kernels
    assert _st(lib, "mck_backward_launch_shape", 4, 8, 1, None) == 1


def test_noalloc_backward_refuses_oversized_problem_without_gpu(lib):
    # the adjoint without allocation: its temporaries must fit the static
    # scratch; 256 row blocks x E = 64 x 3n floats of partial sums (about
    # 200 MB) are refused on the host, before any GPU call
    p16 = ctypes.c_void_p(16)
    fn = "mck_fastfood_backward_p_noalloc"
    assert _st(lib, fn, p16, p16, 8192, 1024, 1024, 64, p16, p16, p16, p16, p16, p16, p16, p16, None) == 2
    assert b"static scratch" in lib.mck_last_error()
    # ... while dx alone needs only the parameter copies: validation passes
    # up to the GPU, which is not touched here (NULL x is refused first)
    assert _st(lib, fn, None, p16, 8192, 1024, 1024, 64, p16, p16, p16, p16, p16, None, None, None, None) == 1
    assert _st(lib, fn, p16, p16, 8192, 1024, 512, 64, p16, p16, p16, p16, p16, p16, p16, p16, None) == 1
    assert _st(lib, fn, p16, p16, 0, 1024, 1024, 64, p16, p16, p16, p16, None, None, None, None, None) == 0
