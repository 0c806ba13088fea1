"""Autograd adjoint of the HIP library against the oracle: energy gradients,
upstream gradients of the field outputs, gradcheck, and the once-differentiable
guard."""
import numpy as np
import pytest
import torch

from oracle.oracle import oracle_ewald
from paper_2408_03273_amd import workloads as wl
from paper_2408_03273_amd.ewald import ewald
from tests import _harness as H

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _leaves(s):
    dev = torch.device("cuda", 0)
    return [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev, requires_grad=True)
            for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]


def test_energy_gradients_match_oracle():
    s = wl.random_system(21, 9, 2345, alpha=0.3, rcut=8.5, kmax=9, neutral=False)
    print(f"[autograd] nq={s.nq} nm={s.nm}", flush=True)
    plan = H.make_plan(s)
    x = _leaves(s)
    E, phi, efield, efgrad = ewald(plan, *x)
    E.backward()
    ref = H.oracle_outputs(s)
    got = dict(g_qm_pos=x[0].grad, g_Q=x[1].grad, g_mu=x[2].grad, g_theta=x[3].grad, g_mm_pos=x[4].grad,
               g_mm_q=x[5].grad)
    errs = {k: H.relerr(v.cpu().numpy(), ref[k]) for k, v in got.items()}
    assert max(errs.values()) <= TOL, errs


def test_upstream_gradients_of_field_outputs():
    """L = a E + g_phi.phi + g_F.efield + g_G.efgrad.  By linearity of the QM-MM
    energy in the moments, the oracle evaluates L's gradient exactly: the
    QM-QM part scaled by a plus the QM-MM part with moments
    (a Q + g_phi, a mu - g_F, a theta - (2,1,1,2,1,2) g_G)."""
    s = wl.random_system(22, 7, 1800, alpha=0.32, rcut=8.0, kmax=8, neutral=False)
    plan = H.make_plan(s)
    x = _leaves(s)
    rng = np.random.default_rng(5)
    a = 0.7
    gphi, gF, gG = rng.normal(size=s.nq), rng.normal(size=(s.nq, 3)), rng.normal(size=(s.nq, 6))
    dev = x[0].device
    E, phi, efield, efgrad = ewald(plan, *x)
    L = (a * E + (torch.tensor(gphi, device=dev) * phi).sum() + (torch.tensor(gF, device=dev) * efield).sum()
         + (torch.tensor(gG, device=dev) * efgrad).sum())
    L.backward()
    mult = np.array([2, 1, 1, 2, 1, 2.0])
    full = oracle_ewald(s.box, s.alpha, s.rcut, s.kmax, s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)
    qmmm_only = oracle_ewald(s.box, s.alpha, s.rcut, s.kmax, s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q, qmqm=False)
    eff = oracle_ewald(s.box, s.alpha, s.rcut, s.kmax, s.qm_pos, a * s.Q + gphi, a * s.mu - gF,
                       a * s.theta - mult * gG, s.mm_pos, s.q, qmqm=False)
    ref = dict(g_qm_pos=a * (full.g_qm_pos - qmmm_only.g_qm_pos) + eff.g_qm_pos,
               g_Q=a * full.g_Q, g_mu=a * full.g_mu, g_theta=a * full.g_theta,
               g_mm_pos=eff.g_mm_pos, g_mm_q=eff.g_mm_q)
    got = dict(g_qm_pos=x[0].grad, g_Q=x[1].grad, g_mu=x[2].grad, g_theta=x[3].grad, g_mm_pos=x[4].grad,
               g_mm_q=x[5].grad)
    errs = {k: H.relerr(v.cpu().numpy(), ref[k]) for k, v in got.items()}
    assert max(errs.values()) <= TOL, errs
    # an independent spot check by central differences of the oracle's L
    def L_oracle(qm, mm):
        r = oracle_ewald(s.box, s.alpha, s.rcut, s.kmax, qm, s.Q, s.mu, s.theta, mm, s.q)
        return (a * r.E + gphi @ r.phi + (gF * -r.dphi).sum() + (gG * (-2 * r.hphi)).sum())
    h = 1e-4
    for (arr_name, i, c) in (("qm", 2, 1), ("mm", 17, 0), ("mm", 1000, 2)):
        qm, mm = s.qm_pos.copy(), s.mm_pos.copy()
        vals = []
        for st in (-2, -1, 1, 2):
            q2, m2 = qm.copy(), mm.copy()
            (q2 if arr_name == "qm" else m2)[i, c] += st * h
            vals.append(L_oracle(q2, m2))
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        g = (x[0] if arr_name == "qm" else x[4]).grad[i, c].item()
        assert abs(g - fd) <= 1e-7 * max(1.0, abs(fd)), (arr_name, i, c, g, fd)


def test_gradcheck_tiny():
    s = wl.random_system(23, 2, 7, box=(9.0, 9.0, 9.0), alpha=0.6, rcut=4.4, kmax=4, neutral=False)
    plan = H.make_plan(s)
    x = _leaves(s)

    def f(*args):
        E, phi, efield, efgrad = ewald(plan, *args)
        return E, phi, efield, efgrad

    assert torch.autograd.gradcheck(f, tuple(x), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_double_backward_raises():
    s = wl.random_system(24, 2, 10, box=(9.0, 9.0, 9.0), alpha=0.6, rcut=4.4, kmax=3)
    plan = H.make_plan(s)
    x = _leaves(s)
    E = ewald(plan, *x)[0]
    (g,) = torch.autograd.grad(E, x[0], create_graph=True)
    with pytest.raises(RuntimeError):
        g.sum().backward()


def test_recompute_adjoint_matches_stored_gradients():
    """ewald_backward with explicit zero field gradients re-runs the adjoint;
    it must agree with the gradients the forward call stored."""
    s = wl.random_system(25, 8, 2222, alpha=0.3, rcut=8.5, kmax=(8, 9, 7), neutral=False)
    plan = H.make_plan(s)
    d = H.to_dev(s)
    args = (d["qm_pos"], d["Q"], d["mu"], d["theta"], d["mm_pos"], d["mm_q"])
    E, phi, ef, eg, ctx = plan.forward(*args, want_ctx=True)
    gE = torch.tensor(1.7, dtype=torch.float64, device=E.device)
    fast = plan.backward(ctx, *args, gE=gE)
    slow = plan.backward(ctx, *args, gE=gE, g_phi=torch.zeros_like(phi), g_efield=torch.zeros_like(ef),
                         g_efgrad=torch.zeros_like(eg))
    torch.cuda.synchronize()
    for a, b, name in zip(fast, slow, H.BWD_KEYS):
        err = H.relerr(a.cpu().numpy(), b.cpu().numpy())
        assert err <= 1e-12, (name, err)
