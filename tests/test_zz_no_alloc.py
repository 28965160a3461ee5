"""The allocation-free dot product (cbct_dot_noalloc) against cbct_dot.

Both run the same kernels in the same order, so their results must be
bitwise equal; the fixed per-device partial-sum array keeps the previous
call's contents, so two calls in a row (the second on a smaller input) check
that nothing stale leaks into a result."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    from paper_2512_21180_amd import cbct
    torch.cuda.set_device(0)
    return cbct


def test_dot_noalloc_equals_dot_on_two_calls(cb):
    gen = torch.Generator(device="cpu").manual_seed(2024)
    for n in (5_000_003, 70_001):      # the second call is on a smaller input
        a = torch.randn(n, generator=gen).cuda()
        b = (torch.rand(n, generator=gen) - 0.25).cuda()
        ws = cb.dot_workspace(n, "cuda")
        ref = torch.zeros(1, dtype=torch.float64, device="cuda")
        got = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        cb.dot(a, b, ws, ref)
        cb.dot_noalloc(a, b, got)
        torch.cuda.synchronize()
        print(f"n={n}: dot {ref.item()!r} noalloc {got.item()!r}", flush=True)
        assert got.item() == ref.item()
        exact = float(np.dot(a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)))
        assert abs(got.item() - exact) <= 1e-12 * float(np.sum(np.abs(
            a.cpu().numpy().astype(np.float64) * b.cpu().numpy().astype(np.float64))))


def test_dot_noalloc_tiny_and_empty(cb):
    # n smaller than one block, and n = 0: every partial cell is rewritten
    for n, want in ((5, 15.0), (0, 0.0)):
        a = torch.arange(1, n + 1, dtype=torch.float32, device="cuda") if n else \
            torch.empty(0, dtype=torch.float32, device="cuda")
        b = torch.ones_like(a)
        got = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        lib = cb.lib()
        st = lib.cbct_dot_noalloc(n, ctypes.c_void_p(a.data_ptr() or 1), ctypes.c_void_p(b.data_ptr() or 1),
                                  ctypes.c_void_p(got.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert st == 0 and got.item() == want


def test_dot_noalloc_rejects_null(cb):
    lib = cb.lib()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert lib.cbct_dot_noalloc(10, None, None, ctypes.c_void_p(out.data_ptr()), None) == -1
    assert lib.cbct_dot_noalloc_max_cells() == 1024
