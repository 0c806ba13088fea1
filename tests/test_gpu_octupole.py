"""Charge-octupole error estimate and R_cut pick on the GPU against the
oracle: several candidate chunks, spheres beyond the cell, the full c3 size,
and the empty cases."""
import numpy as np
import pytest
import torch

from oracle.oracle import oracle_octupole_error, oracle_rcut_pick
from paper_2408_03273_amd import workloads as wl
from tests import _harness as H

pytestmark = pytest.mark.gpu


def _omega(seed, nq, scale=0.05):
    return np.random.default_rng(seed).normal(0.0, scale, (nq, 10))


def _run(s, omega, r_first, r_step, n_r, r_outer, eps):
    plan = H.make_plan(s)
    d = H.to_dev(s)
    om = torch.tensor(omega, dtype=torch.float64, device=d["Q"].device)
    err, rc = plan.octupole_error(d["qm_pos"], om, d["mm_pos"], d["mm_q"], r_first, r_step, n_r, r_outer, eps)
    torch.cuda.synchronize()
    return err.cpu().numpy(), float(rc.item())


def _check(s, omega, r_first, r_step, n_r, r_outer, eps_quantile=0.5):
    cands = r_first + r_step * np.arange(n_r)
    ref = oracle_octupole_error(s.box, s.qm_pos, omega, s.mm_pos, s.q, cands, r_outer)
    # a threshold between two of the estimates, so the pick is not decided by rounding
    srt = np.sort(np.abs(ref))
    m = min(int(eps_quantile * n_r), n_r - 2) if n_r > 1 else 0
    eps = float(np.sqrt(srt[m] * srt[m + 1])) if n_r > 1 and srt[m] > 0 else 1e-3
    got, rc = _run(s, omega, r_first, r_step, n_r, r_outer, eps)
    scale = float(np.max(np.abs(ref)))
    print(f"[octupole] nq={s.nq} nm={s.nm} n_r={n_r} max|err|={scale:.3e} eps={eps:.3e} r_cut={rc}", flush=True)
    assert np.max(np.abs(got - ref)) <= 1e-10 * scale, (got, ref)
    big = np.abs(ref) > 1e-3 * scale
    assert np.all(np.abs(got[big] - ref[big]) <= 1e-9 * np.abs(ref[big]))
    assert rc == oracle_rcut_pick(cands, ref, eps)


@pytest.mark.parametrize("case", [
    (71, 10, 3000, (24.0, 25.0, 26.0), 4.0, 1.0, 20, 22.0),    # two candidate chunks, sphere past half the box
    (72, 25, 4200, (30.0, 30.0, 30.0), 8.0, 0.5, 40, 35.0),    # three chunks, 17 QM sites per tile row
    (73, 3, 700, (12.4, 12.4, 12.4), 2.0, 2.0, 7, 40.0),       # r_outer above three box lengths
])
def test_octupole_parity(case):
    seed, nq, nm, box, r_first, r_step, n_r, r_outer = case
    s = wl.random_system(seed, nq, nm, box=box, neutral=True)
    _check(s, _omega(seed, nq), r_first, r_step, n_r, r_outer)


def test_octupole_c3_size():
    s = wl.random_system(74, 40, 35000, box=(70.0, 70.0, 72.0), neutral=True)
    _check(s, _omega(74, 40), 10.0, 2.0, 12, 34.0, eps_quantile=0.3)


def test_octupole_empty_cases():
    s = wl.random_system(75, 4, 0, box=(20.0, 20.0, 20.0))
    got, rc = _run(s, _omega(75, 4), 5.0, 1.0, 5, 9.0, 1e-6)
    assert np.all(got == 0.0) and rc == 5.0
    s = wl.random_system(76, 4, 50, box=(20.0, 20.0, 20.0))
    got, rc = _run(s, _omega(76, 4), 5.0, 1.0, 1, 9.0, 1e-6)  # one candidate: no consecutive pair
    assert rc == -1.0


def test_octupole_no_qm_sites():
    s = wl.random_system(77, 0, 40, box=(20.0, 20.0, 20.0))
    got, rc = _run(s, np.zeros((0, 10)), 3.0, 1.0, 4, 9.0, 1e-6)
    assert np.all(got == 0.0) and rc == 3.0
