"""Helpers shared by the GPU tests: run the HIP library and the oracle on the
same seeded System and compare every output array normwise."""
from __future__ import annotations

import numpy as np

from oracle.oracle import oracle_ewald

FWD_KEYS = ("energy", "phi", "efield", "efgrad")
BWD_KEYS = ("g_qm_pos", "g_Q", "g_mu", "g_theta", "g_mm_pos", "g_mm_q")


def relerr(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError(f"shape mismatch {a.shape} vs {b.shape}")
    if a.size == 0:
        return 0.0
    den = float(np.max(np.abs(b)))
    num = float(np.max(np.abs(a - b)))
    return num / den if den > 0 else num


def oracle_outputs(sys, qmqm=True, mm_sel=None) -> dict:
    r = oracle_ewald(sys.box, sys.alpha, sys.rcut, sys.kmax, sys.qm_pos, sys.Q, sys.mu, sys.theta, sys.mm_pos, sys.q,
                     qmqm=qmqm, mm_sel=mm_sel)
    return dict(energy=np.array(r.E), phi=r.phi, efield=-r.dphi, efgrad=-2.0 * r.hphi, g_qm_pos=r.g_qm_pos, g_Q=r.g_Q,
                g_mu=r.g_mu, g_theta=r.g_theta, g_mm_pos=r.g_mm_pos, g_mm_q=r.g_mm_q, _raw=r)


def to_dev(sys, device="cuda"):
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)  # noqa: E731
    return dict(qm_pos=t(sys.qm_pos.reshape(-1, 3)), Q=t(sys.Q), mu=t(sys.mu.reshape(-1, 3)),
                theta=t(sys.theta.reshape(-1, 6)), mm_pos=t(sys.mm_pos.reshape(-1, 3)), mm_q=t(sys.q))


def make_plan(sys, qmqm=True, precision="fp64", plain=False, max_qm=None, max_mm=None, max_frames=1, cell_list=True):
    from paper_2408_03273_amd.ewald import EwaldConfig, Plan
    cfg = EwaldConfig(box=tuple(sys.box), alpha=sys.alpha, rcut=sys.rcut, kmax=tuple(sys.kmax),
                      max_qm=max_qm if max_qm is not None else max(sys.nq, 1),
                      max_mm=max_mm if max_mm is not None else max(sys.nm, 1), max_frames=max_frames, qmqm=qmqm,
                      precision=precision, plain=plain, cell_list=cell_list)
    return Plan(cfg)


def gpu_outputs(sys, plan=None, backward=True, **kw) -> dict:
    import torch
    plan = plan or make_plan(sys, **kw)
    d = to_dev(sys)
    energy, phi, efield, efgrad, ctx = plan.forward(d["qm_pos"], d["Q"], d["mu"], d["theta"], d["mm_pos"], d["mm_q"],
                                                    want_ctx=backward)
    out = dict(energy=energy, phi=phi, efield=efield, efgrad=efgrad)
    if backward:
        g = plan.backward(ctx, d["qm_pos"], d["Q"], d["mu"], d["theta"], d["mm_pos"], d["mm_q"])
        out.update(zip(BWD_KEYS, g))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def compare(gpu: dict, ref: dict, keys, mm_sel=None) -> dict:
    errs = {}
    for k in keys:
        a = gpu[k]
        if mm_sel is not None and k in ("g_mm_pos", "g_mm_q"):
            a = a[mm_sel]
        errs[k] = relerr(a, ref[k])
    return errs
