"""The C ABI library loads, exports every function its header declares, and
rejects bad arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2408_03273_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpewald.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ewald_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    fns = header_functions()
    for name in ("ewald_setup", "ewald_forward", "ewald_backward", "ewald_batch"):
        assert name in fns
    assert set(fns) == set(_lib.EXPORTED), f"binding list out of date: {set(fns) ^ set(_lib.EXPORTED)}"


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [f for f in header_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_version_and_last_error_strings():
    lib = _lib.load()
    assert lib.ewald_version().decode().startswith("mpewald")
    assert isinstance(lib.ewald_last_error(), bytes)


def _params(**kw):
    p = _lib.EwaldParams()
    p.box[:] = kw.get("box", (20.0, 20.0, 20.0))
    p.alpha = kw.get("alpha", 0.3)
    p.rcut = kw.get("rcut", 9.0)
    p.kmax[:] = kw.get("kmax", (8, 8, 8))
    p.precision = kw.get("precision", 0)
    p.flags = kw.get("flags", 1)
    p.max_qm, p.max_mm, p.max_frames = kw.get("caps", (10, 100, 1))
    return p


@pytest.mark.parametrize("kw,status", [
    (dict(alpha=0.0), _lib.EWALD_ERR_ARG),
    (dict(alpha=-1.0), _lib.EWALD_ERR_ARG),
    (dict(rcut=0.0), _lib.EWALD_ERR_ARG),
    # more than 3 lattice images per direction beyond the minimum image
    (dict(rcut=75.0), _lib.EWALD_ERR_CUTOFF),
    (dict(box=(20.0, 15.0, 20.0), rcut=55.0), _lib.EWALD_ERR_CUTOFF),
    (dict(kmax=(0, 8, 8)), _lib.EWALD_ERR_ARG),
    (dict(box=(20.0, -1.0, 20.0)), _lib.EWALD_ERR_ARG),
    (dict(precision=7), _lib.EWALD_ERR_ARG),
    (dict(precision=4), _lib.EWALD_ERR_ARG),
    (dict(precision=-1), _lib.EWALD_ERR_ARG),
    (dict(flags=1 << 10), _lib.EWALD_ERR_ARG),
    (dict(caps=(10, 100, 0)), _lib.EWALD_ERR_ARG),
])
def test_setup_rejects_bad_parameters(kw, status):
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.ewald_setup(ctypes.byref(_params(**kw)), ctypes.byref(h))
    assert st == status, (st, lib.ewald_last_error())
    assert lib.ewald_last_error().decode() != ""
    assert not h.value


def test_null_arguments_rejected():
    lib = _lib.load()
    assert lib.ewald_setup(None, None) == _lib.EWALD_ERR_ARG
    z = [None] * 13
    assert lib.ewald_forward(None, 0, *z[:4], 0, *z[:2], *z[:5], None) == _lib.EWALD_ERR_ARG
    assert lib.ewald_backward(None, None, 0, *[None] * 4, 0, *[None] * 2, *[None] * 10, None) == _lib.EWALD_ERR_ARG
    assert lib.ewald_batch(None, 1, None, *[None] * 6, 0, *[None] * 10, None) == _lib.EWALD_ERR_ARG
    assert lib.ewald_destroy(None) == _lib.EWALD_OK
    assert lib.ewald_ctx_bytes(None, 1, 1) == 0


def test_no_cpu_fallback_in_product_path():
    """The Python front-end must refuse to run without a GPU rather than fall back."""
    import torch
    from paper_2408_03273_amd.ewald import EwaldConfig, Plan
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        Plan(EwaldConfig(box=(20, 20, 20), alpha=0.3, rcut=9, kmax=8, max_qm=1, max_mm=1))


def test_noalloc_octupole_host_checks():
    """The allocation-free octupole estimate validates on the host before any
    device call: a null box, bad candidates and more partial sums than its
    fixed device array holds are refused (the pointers are never read)."""
    lib = _lib.load()
    box = (ctypes.c_double * 3)(20.0, 20.0, 20.0)
    fake = ctypes.c_void_p(0x1000)
    assert lib.ewald_octupole_error_noalloc(None, 2, fake, fake, 10, fake, fake, 4, 1.0, 1.0, 9.0, 1e-3, fake, None,
                                            None) == _lib.EWALD_ERR_ARG
    assert lib.ewald_octupole_error_noalloc(box, 2, fake, fake, 10, fake, fake, 0, 1.0, 1.0, 9.0, 1e-3, fake, None,
                                            None) == _lib.EWALD_ERR_ARG
    assert lib.ewald_octupole_error_noalloc(box, 2, fake, fake, 10, fake, fake, 4, 1.0, 1.0, 90.0, 1e-3, fake, None,
                                            None) == _lib.EWALD_ERR_CUTOFF
    assert lib.ewald_octupole_error_noalloc(box, 2, fake, fake, 1100000, fake, fake, 256, 1.0, 0.1, 30.0, 1e-3, fake,
                                            None, None) == _lib.EWALD_ERR_CAPACITY
