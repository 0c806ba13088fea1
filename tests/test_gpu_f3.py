"""The paper's parameter regime (Computational Details: a real-space cutoff of
about the box length, Ewald parameters for a target accuracy): rc = 0.95 of
the smallest box edge, alpha and kmax from ewald_suggest_params at 1e-8, so
real space sums up to 27 lattice images per pair and the k-set is small.
GPU against the oracle through autograd (every output; at the c3 size the MM
gradients on a sample of rows), and the FP32 real-space variant's error."""
import numpy as np
import pytest
import torch

from oracle.oracle import oracle_ewald
from paper_2408_03273_amd import workloads as wl
from paper_2408_03273_amd.ewald import EwaldConfig, Plan, ewald, suggest_params
from tests import _harness as H

pytestmark = pytest.mark.gpu
ALL = H.FWD_KEYS + H.BWD_KEYS


def f3_system(s, frac=0.95, tol=1e-8):
    """s with rc = frac * min(box) and alpha, kmax for the accuracy tol."""
    rc = frac * float(np.min(s.box))
    alpha, kmax = suggest_params(s.box, rc, tol)
    return wl.System(box=s.box, alpha=alpha, rcut=rc, kmax=kmax, qm_pos=s.qm_pos, Q=s.Q, mu=s.mu, theta=s.theta,
                     mm_pos=s.mm_pos, q=s.q, name=s.name + "/f3")


def _autograd(s, precision="fp64"):
    dev = torch.device("cuda", 0)
    plan = Plan(EwaldConfig(box=tuple(s.box), alpha=s.alpha, rcut=s.rcut, kmax=tuple(s.kmax), max_qm=s.nq,
                            max_mm=s.nm, precision=precision))
    x = [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev, requires_grad=True)
         for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]
    E, phi, efield, efgrad = ewald(plan, *x)
    E.backward()
    torch.cuda.synchronize()
    out = [E, phi, efield, efgrad] + [t.grad for t in x]
    return dict(zip(ALL, (t.detach().cpu().numpy() for t in out)))


def test_f3_small_full_parity():
    s = f3_system(wl.random_system(401, 12, 3000, box=(20.0, 21.0, 22.0), neutral=False))
    print(f"[f3] {s.name}: rc={s.rcut:.2f} alpha={s.alpha:.4f} kmax={s.kmax}", flush=True)
    errs = H.compare(_autograd(s), H.oracle_outputs(s), ALL)
    print(f"[f3] worst {max(errs.values()):.2e}", flush=True)
    assert max(errs.values()) <= 1e-10, errs


def test_f3_c3_size():
    s = f3_system(wl.make_config(3))
    sel = np.arange(0, s.nm, 97)
    r = oracle_ewald(s.box, s.alpha, s.rcut, s.kmax, s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q, mm_sel=sel)
    ref = dict(energy=np.array(r.E), phi=r.phi, efield=-r.dphi, efgrad=-2.0 * r.hphi, g_qm_pos=r.g_qm_pos, g_Q=r.g_Q,
               g_mu=r.g_mu, g_theta=r.g_theta, g_mm_pos=r.g_mm_pos, g_mm_q=r.g_mm_q)
    got = _autograd(s)
    errs = H.compare(got, ref, ALL, mm_sel=sel)
    print(f"[f3] c3: rc={s.rcut} alpha={s.alpha:.4f} kmax={s.kmax} worst {max(errs.values()):.2e}", flush=True)
    assert max(errs.values()) <= 1e-10, errs
    # FP32 real space with FP64 accumulation: error reported (not a parity gate)
    g32 = _autograd(s, "fp32_real")
    e32 = H.compare(g32, got, ALL)
    print("[f3] FP32 real space vs FP64:", {k: f"{v:.1e}" for k, v in e32.items()}, flush=True)
    assert max(e32.values()) < 1e-4


def test_f3_full_backward_path():
    """The backward pass that takes upstream gradients on the per-site outputs
    (zero here, so it must reproduce the gradients of E): real space's MM side
    from the per-atom kernel over site groups."""
    s = f3_system(wl.random_system(402, 17, 2600, box=(21.0, 20.0, 23.0), neutral=False))
    plan = H.make_plan(s)
    d = H.to_dev(s)
    args = (d["qm_pos"], d["Q"], d["mu"], d["theta"], d["mm_pos"], d["mm_q"])
    energy, phi, ef, efg, ctx = plan.forward(*args, want_ctx=True)
    g = plan.backward(ctx, *args, gE=torch.ones((), dtype=torch.float64, device=plan.device),
                      g_phi=torch.zeros_like(phi), g_efield=torch.zeros_like(ef), g_efgrad=torch.zeros_like(efg))
    torch.cuda.synchronize()
    got = dict(zip(H.BWD_KEYS, (t.cpu().numpy() for t in g)))
    errs = H.compare(got, H.oracle_outputs(s), H.BWD_KEYS)
    print(f"[f3] full backward path worst {max(errs.values()):.2e}", flush=True)
    assert max(errs.values()) <= 1e-10, errs


def _f3_frames():
    base = [wl.random_system(410 + i, nq, nm, box=box, neutral=False)
            for i, (nq, nm, box) in enumerate([(14, 2200, (20.0, 21.0, 22.0)), (9, 3100, (22.5, 22.0, 23.0)),
                                               (21, 1500, (19.5, 20.5, 20.0))])]
    rc = 0.95 * min(float(np.min(b.box)) for b in base)
    alpha, kmax = suggest_params(base[2].box, rc, 1e-8)
    return [wl.System(box=b.box, alpha=alpha, rcut=rc, kmax=kmax, qm_pos=b.qm_pos, Q=b.Q, mu=b.mu, theta=b.theta,
                      mm_pos=b.mm_pos, q=b.q, name=b.name + "/f3") for b in base]


def _batch(frames, deterministic=False, calls=1):
    qoff = np.cumsum([0] + [f.nq for f in frames])
    moff = np.cumsum([0] + [f.nm for f in frames])
    desc = [dict(box=f.box, n_qm=f.nq, n_mm=f.nm, qm_offset=int(qoff[i]), mm_offset=int(moff[i]))
            for i, f in enumerate(frames)]
    dev = torch.device("cuda", 0)
    cat = lambda k: torch.tensor(np.concatenate([getattr(f, k) for f in frames]), dtype=torch.float64,  # noqa: E731
                                 device=dev)
    x = [cat("qm_pos"), cat("Q"), cat("mu"), cat("theta"), cat("mm_pos"), cat("q")]
    f0 = frames[0]
    plan = Plan(EwaldConfig(box=tuple(f0.box), alpha=f0.alpha, rcut=f0.rcut, kmax=tuple(f0.kmax), max_qm=int(qoff[-1]),
                            max_mm=int(moff[-1]), max_frames=len(frames), deterministic=deterministic))
    outs = []
    for _ in range(calls):
        o = plan.batch(desc, *x)
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in o.items()})
    plan.close()

    def frame_out(o, i):
        sq, sm = slice(qoff[i], qoff[i + 1]), slice(moff[i], moff[i + 1])
        return dict(energy=o["energy"][i], phi=o["phi"][sq], efield=o["efield"][sq], efgrad=o["efgrad"][sq],
                    g_qm_pos=o["g_qm_pos"][sq], g_Q=o["g_Q"][sq], g_mu=o["g_mu"][sq], g_theta=o["g_theta"][sq],
                    g_mm_pos=o["g_mm_pos"][sm], g_mm_q=o["g_mm_q"][sm])
    return outs, frame_out


@pytest.mark.parametrize("deterministic", [False, True])
def test_f3_batch_frames(deterministic):
    """Three frames of different boxes and sizes in one batched call, each in
    full against the oracle; deterministic plans also bitwise repeatable."""
    frames = _f3_frames()
    outs, frame_out = _batch(frames, deterministic, calls=2 if deterministic else 1)
    for i, f in enumerate(frames):
        errs = H.compare(frame_out(outs[0], i), H.oracle_outputs(f), ALL)
        print(f"[f3] batch frame {i} (det={deterministic}) worst {max(errs.values()):.2e}", flush=True)
        assert max(errs.values()) <= 1e-10, (i, errs)
    if deterministic:
        for k in outs[0]:
            assert np.array_equal(outs[0][k], outs[1][k]), k
