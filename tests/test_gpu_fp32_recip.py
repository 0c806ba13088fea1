"""Mixed-precision variant: the two reciprocal-space hot loops on FP32 matrix
cores (phase tables and folded weights rounded to FP32, FP64 sums across
blocks).  Its error against the FP64 oracle is reported and bounded by a
tolerance derived from FP32 rounding: unit roundoff u = 6e-8 on each table
entry and a random-walk accumulation over at most ~10^3 terms inside a block
give about u sqrt(1e3) = 2e-6 relative on S(k), the energy and the forces;
the bound is 2.5 times that (measured: at most 6e-7)."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2408_03273_amd import workloads as wl
from paper_2408_03273_amd.ewald import EwaldConfig, Plan, ewald
from tests import _harness as H

pytestmark = pytest.mark.gpu
TOL32 = 5e-6
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _run(s, precision, dev):
    x = [torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True)
         for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]
    plan = Plan(EwaldConfig(box=tuple(s.box), alpha=s.alpha, rcut=s.rcut, kmax=s.kmax, max_qm=s.nq, max_mm=s.nm,
                            precision=precision))
    E, phi, efield, efgrad = ewald(plan, *x)
    E.backward()
    torch.cuda.synchronize()
    out = dict(energy=E.item(), phi=phi.detach().cpu().numpy(), efield=efield.detach().cpu().numpy(),
               efgrad=efgrad.detach().cpu().numpy(), g_qm_pos=x[0].grad.cpu().numpy(), g_Q=x[1].grad.cpu().numpy(),
               g_mu=x[2].grad.cpu().numpy(), g_theta=x[3].grad.cpu().numpy(), g_mm_pos=x[4].grad.cpu().numpy(),
               g_mm_q=x[5].grad.cpu().numpy())
    return out, plan.describe()


def test_fp32_recip_c3_against_oracle():
    s = wl.make_config(3)
    with open(os.path.join(GOLDEN, "oracle_c3_f0.json")) as f:
        g = json.load(f)
    assert s.sha256() == g["input_sha256"]
    got, desc = _run(s, "fp32_recip", torch.device("cuda", 0))
    assert "fp32-recip" in desc
    sel = np.array(g["mm_sel"])
    errs = {}
    for k in H.FWD_KEYS + H.BWD_KEYS:
        a = np.asarray(got[k])
        if k in ("g_mm_pos", "g_mm_q"):
            a = a[sel]
        errs[k] = H.relerr(a, np.asarray(g[k]))
    print("[fp32-recip] c3 relative errors vs the FP64 oracle:", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= TOL32, errs
    # it is a different computation: not bit-identical to the FP64 path
    assert max(errs.values()) > 1e-12


@pytest.mark.parametrize("case", [(81, 17, 3000, (21.0, 22.0, 23.0), 0.33, 9.0, (8, 9, 10)),
                                  (82, 5, 700, (17.0, 17.0, 17.0), 0.4, 8.0, (5, 5, 3)),
                                  # |ny| <= 33: a large y grid (35 KB of FP32 y rows per 64-atom block)
                                  (83, 6, 1501, (18.0, 20.0, 22.0), 0.35, 8.0, (5, 33, 9))])
def test_fp32_recip_small_against_oracle(case):
    seed, nq, nm, box, alpha, rcut, kmax = case
    s = wl.random_system(seed, nq, nm, box=box, alpha=alpha, rcut=rcut, kmax=kmax, neutral=False)
    ref = H.oracle_outputs(s)
    got, _ = _run(s, "fp32_recip", torch.device("cuda", 0))
    errs = H.compare({k: np.asarray(v) for k, v in got.items()}, ref, H.FWD_KEYS + H.BWD_KEYS)
    print(f"[fp32-recip] seed {seed}:", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= TOL32, errs


def test_fp32_recip_batch_against_oracle():
    """Three c4 frames through ewald_batch with the FP32 hot loops."""
    frames = [wl.make_config(4, f) for f in range(3)]
    qoff = np.cumsum([0] + [f.nq for f in frames])
    moff = np.cumsum([0] + [f.nm for f in frames])
    desc = [dict(box=f.box, n_qm=f.nq, n_mm=f.nm, qm_offset=int(qoff[i]), mm_offset=int(moff[i]))
            for i, f in enumerate(frames)]
    dev = torch.device("cuda", 0)
    cat = lambda k: torch.tensor(np.concatenate([getattr(f, k) for f in frames]), dtype=torch.float64,  # noqa: E731
                                 device=dev)
    f0 = frames[0]
    plan = Plan(EwaldConfig(box=tuple(f0.box), alpha=f0.alpha, rcut=f0.rcut, kmax=f0.kmax, max_qm=int(qoff[-1]),
                            max_mm=int(moff[-1]), max_frames=3, precision="fp32_recip"))
    out = plan.batch(desc, cat("qm_pos"), cat("Q"), cat("mu"), cat("theta"), cat("mm_pos"), cat("q"))
    torch.cuda.synchronize()
    for i in range(3):
        with open(os.path.join(GOLDEN, f"oracle_c4_f{i}.json")) as f:
            g = json.load(f)
        q0, q1, m0 = int(qoff[i]), int(qoff[i + 1]), int(moff[i])
        sel = np.array(g["mm_sel"]) + m0
        got = dict(energy=out["energy"][i].item(), phi=out["phi"][q0:q1].cpu().numpy(),
                   efield=out["efield"][q0:q1].cpu().numpy(), efgrad=out["efgrad"][q0:q1].cpu().numpy(),
                   g_qm_pos=out["g_qm_pos"][q0:q1].cpu().numpy(), g_Q=out["g_Q"][q0:q1].cpu().numpy(),
                   g_mu=out["g_mu"][q0:q1].cpu().numpy(), g_theta=out["g_theta"][q0:q1].cpu().numpy(),
                   g_mm_pos=out["g_mm_pos"].cpu().numpy()[sel], g_mm_q=out["g_mm_q"].cpu().numpy()[sel])
        errs = {k: H.relerr(np.asarray(got[k]), np.asarray(g[k])) for k in H.FWD_KEYS + H.BWD_KEYS}
        print(f"[fp32-recip] c4 frame {i}:", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
        assert max(errs.values()) <= TOL32, (i, errs)


def test_fp32_recip_rejects_grids_without_its_kernels():
    from paper_2408_03273_amd import _lib
    with pytest.raises(_lib.EwaldError) as ei:
        Plan(EwaldConfig(box=(40.0, 40.0, 40.0), alpha=0.3, rcut=9.0, kmax=(8, 8, 40), max_qm=4, max_mm=10,
                         precision="fp32_recip"))
    assert "EWALD_ERR_ARG" in str(ei.value)
    # the FP64 path takes the same grid (VALU kernels)
    Plan(EwaldConfig(box=(40.0, 40.0, 40.0), alpha=0.3, rcut=9.0, kmax=(8, 8, 40), max_qm=4, max_mm=10)).close()
