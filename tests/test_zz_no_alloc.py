"""The allocation-free octupole estimate (no plan; block partial sums in the
library's fixed device array) against the plan entry point on the same
inputs, through the C ABI: a large call, then a smaller one (the fixed array
still holds the first call's partial sums), then one without MM atoms."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2408_03273_amd import _lib
from paper_2408_03273_amd import workloads as wl
from tests import _harness as H

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _inputs(s, seed):
    d = H.to_dev(s)
    d["omega"] = torch.tensor(np.random.default_rng(seed).normal(0.0, 0.05, (s.nq, 10)), dtype=torch.float64,
                              device=d["Q"].device)
    return d


def _noalloc(s, d, r_first, r_step, n_r, r_outer, eps):
    lib = _lib.load()
    dev = d["Q"].device
    err = torch.full((n_r,), float("nan"), dtype=torch.float64, device=dev)
    rc = torch.full((), float("nan"), dtype=torch.float64, device=dev)
    box = (ctypes.c_double * 3)(*[float(b) for b in s.box])
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _lib.check(lib.ewald_octupole_error_noalloc(box, s.nq, _p(d["qm_pos"]), _p(d["omega"]), s.nm, _p(d["mm_pos"]),
                                                _p(d["mm_q"]), n_r, r_first, r_step, r_outer, eps, _p(err), _p(rc),
                                                stream))
    torch.cuda.synchronize()
    return err.cpu().numpy(), float(rc.item())


def _with_plan(s, d, r_first, r_step, n_r, r_outer, eps):
    plan = H.make_plan(s)
    err, rc = plan.octupole_error(d["qm_pos"], d["omega"], d["mm_pos"], d["mm_q"], r_first, r_step, n_r, r_outer, eps)
    torch.cuda.synchronize()
    out = err.cpu().numpy(), float(rc.item())
    plan.close()
    return out


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_octupole_matches_plan_entry_point(order):
    cases = [
        # seed, nq, nm, box, r_first, r_step, n_r, r_outer: 118 MM blocks x 40 candidates, then 12 x 12
        (81, 20, 30000, (40.0, 41.0, 42.0), 6.0, 0.5, 40, 30.0),
        (82, 7, 3000, (22.0, 23.0, 24.0), 4.0, 1.0, 12, 20.0),
    ]
    for seed, nq, nm, box, r_first, r_step, n_r, r_outer in cases:
        s = wl.random_system(seed, nq, nm, box=box, neutral=True)
        d = _inputs(s, seed)
        ref, rc_ref = _with_plan(s, d, r_first, r_step, n_r, r_outer, 1.0)
        srt = np.sort(np.abs(ref))
        eps = float(np.sqrt(srt[n_r // 2] * srt[n_r // 2 + 1]))   # between two estimates: a definite pick
        ref, rc_ref = _with_plan(s, d, r_first, r_step, n_r, r_outer, eps)
        got, rc = _noalloc(s, d, r_first, r_step, n_r, r_outer, eps)
        scale = float(np.max(np.abs(ref)))
        print(f"[noalloc] nq={nq} nm={nm} n_r={n_r} max|err|={scale:.3e} diff={np.max(np.abs(got - ref)):.2e} "
              f"r_cut={rc} (plan {rc_ref})", flush=True)
        assert scale > 0.0
        assert np.max(np.abs(got - ref)) <= 1e-10 * scale
        assert rc == rc_ref
    # no MM atoms: every estimate is zero and the first candidate is picked
    s = wl.random_system(83, 4, 0, box=(20.0, 20.0, 20.0))
    d = _inputs(s, 83)
    got, rc = _noalloc(s, d, 5.0, 1.0, 5, 9.0, 1e-6)
    assert np.all(got == 0.0) and rc == 5.0


def test_noalloc_rejects_too_many_partials():
    s = wl.random_system(84, 2, 10, box=(20.0, 20.0, 20.0))
    d = _inputs(s, 84)
    lib = _lib.load()
    box = (ctypes.c_double * 3)(20.0, 20.0, 20.0)
    err = torch.zeros(256, dtype=torch.float64, device=d["Q"].device)
    # 256 candidates x ceil(1.1e6 / 256) blocks > 2^20: refused on the host, nothing launched
    st = lib.ewald_octupole_error_noalloc(box, s.nq, _p(d["qm_pos"]), _p(d["omega"]), 1100000, _p(d["mm_pos"]),
                                          _p(d["mm_q"]), 256, 1.0, 0.1, 30.0, 1e-3, _p(err), None, None)
    assert st == _lib.EWALD_ERR_CAPACITY
    assert b"allocation-free" in lib.ewald_last_error()
    torch.cuda.synchronize()
    assert float(err.abs().max()) == 0.0
