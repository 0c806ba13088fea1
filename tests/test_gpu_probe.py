"""The FP64 throughput probe (a diagnostic entry point) through the C ABI:
flop count of a launch, finite per-wave values, and argument checks."""
import ctypes

import pytest

from paper_2408_03273_amd import _lib


@pytest.mark.gpu
@pytest.mark.parametrize("kind,per_iter", [(0, 4 * 4 * 2048), (1, 256 * 8 * 2)])
def test_probe_flops_and_outputs(kind, per_iter):
    import torch
    lib = _lib.load()
    blocks, iters = 16, 40
    out = torch.full((4 * blocks,), float("nan"), dtype=torch.float64, device="cuda")
    fl = ctypes.c_double(0.0)
    s = torch.cuda.current_stream()
    st = lib.ewald_fp64_probe(kind, blocks, iters, ctypes.c_void_p(out.data_ptr()), ctypes.byref(fl),
                              ctypes.c_void_p(s.cuda_stream))
    assert st == 0, _lib.load().ewald_last_error()
    torch.cuda.synchronize()
    assert fl.value == float(blocks * per_iter * iters)
    v = out.cpu()
    assert torch.isfinite(v).all()


def test_probe_rejects_bad_arguments():
    lib = _lib.load()
    fl = ctypes.c_double(0.0)
    dummy = ctypes.c_void_p(1)  # never dereferenced: the checks come first
    for kind, blocks, iters in ((2, 1, 1), (-1, 1, 1), (0, 0, 1), (0, 65537, 1), (1, 1, 0), (1, 1, 10000001)):
        assert lib.ewald_fp64_probe(kind, blocks, iters, dummy, ctypes.byref(fl), None) == -1
        assert lib.ewald_last_error()
    assert lib.ewald_fp64_probe(0, 1, 1, None, ctypes.byref(fl), None) == -1
    assert lib.ewald_fp64_probe(0, 1, 1, dummy, None, None) == -1
