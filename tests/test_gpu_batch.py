"""Batched multi-frame path (one HIP-graph replay per call) against unbatched
calls and the oracle; frame order, replays after in-place input changes,
capacity errors."""
import numpy as np
import pytest
import torch

from paper_2408_03273_amd import workloads as wl
from paper_2408_03273_amd._lib import EWALD_ERR_CAPACITY, EwaldError
from paper_2408_03273_amd.ewald import EwaldConfig, Plan
from tests import _harness as H

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _frames(seeds_sizes, alpha=0.3, rcut=8.0, kmax=8):
    out = []
    for seed, nq, nm, L in seeds_sizes:
        out.append(wl.random_system(seed, nq, nm, box=(L, L * 1.05, L * 0.97), alpha=alpha, rcut=rcut, kmax=kmax))
    return out


def _pack(frames, order=None):
    order = list(range(len(frames))) if order is None else order
    fr = [frames[i] for i in order]
    qoff = np.cumsum([0] + [f.nq for f in fr])
    moff = np.cumsum([0] + [f.nm for f in fr])
    desc = [dict(box=f.box, n_qm=f.nq, n_mm=f.nm, qm_offset=int(qoff[i]), mm_offset=int(moff[i]))
            for i, f in enumerate(fr)]
    cat = lambda k, w: torch.tensor(np.concatenate([getattr(f, k).reshape(-1, w) for f in fr]).reshape(  # noqa: E731
        (-1,) if w == 1 else (-1, w)), dtype=torch.float64, device=DEV)
    x = [cat("qm_pos", 3), cat("Q", 1), cat("mu", 3), cat("theta", 6), cat("mm_pos", 3), cat("q", 1)]
    return desc, x, qoff, moff


def _batch_plan(frames, max_frames=None):
    f0 = frames[0]
    return Plan(EwaldConfig(box=tuple(f0.box), alpha=f0.alpha, rcut=f0.rcut, kmax=f0.kmax,
                            max_qm=sum(f.nq for f in frames), max_mm=sum(f.nm for f in frames),
                            max_frames=max_frames or len(frames)))


FRAMES = [(31, 12, 3001, 20.0), (32, 5, 517, 17.5), (33, 23, 4444, 22.0), (34, 1, 1200, 18.0), (35, 17, 2048, 19.0),
          (36, 9, 0, 18.5)]


def _per_frame(frames, out, qoff, moff, i):
    sl_q, sl_m = slice(qoff[i], qoff[i + 1]), slice(moff[i], moff[i + 1])
    o = {k: v.cpu().numpy() for k, v in out.items()}
    return dict(energy=o["energy"][i], phi=o["phi"][sl_q], efield=o["efield"][sl_q], efgrad=o["efgrad"][sl_q],
                g_qm_pos=o["g_qm_pos"][sl_q], g_Q=o["g_Q"][sl_q], g_mu=o["g_mu"][sl_q],
                g_theta=o["g_theta"][sl_q], g_mm_pos=o["g_mm_pos"][sl_m], g_mm_q=o["g_mm_q"][sl_m])


def test_batch_matches_unbatched_and_oracle():
    frames = _frames(FRAMES)
    desc, x, qoff, moff = _pack(frames)
    plan = _batch_plan(frames)
    out = plan.batch(desc, *x)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        print(f"[batch] frame {i}: nq={f.nq} nm={f.nm}", flush=True)
        got = _per_frame(frames, out, qoff, moff, i)
        single = H.gpu_outputs(f)
        keys = H.FWD_KEYS + H.BWD_KEYS
        errs = H.compare(got, single, keys)
        assert max(errs.values()) <= 1e-12, (i, errs)
        if i < 3:
            ref = H.oracle_outputs(f)
            errs = H.compare(got, ref, keys)
            assert max(errs.values()) <= 1e-10, (i, errs)


@pytest.mark.parametrize("fwd_xcd,target,one_stream", [("0", "64", "0"), ("1", "64", "1"), ("1", "65536", "0"),
                                                        ("0", "65536", "1")])
def test_batch_schedules_agree(monkeypatch, fwd_xcd, target, one_stream):
    """The batch's forward block orders (frame-major grid, or the XCD-aware
    one-dimensional grid over (frame, atom chunk) units), its chunk sizes (896
    atoms, a few per frame with ragged last ones, or 64, which divide the
    2048-atom frame exactly; the frame without MM atoms owns none) and its one-
    or two-stream schedule give the single-frame results of every frame."""
    monkeypatch.setenv("MPEWALD_FWD_XCD", fwd_xcd)
    monkeypatch.setenv("MPEWALD_BATCH_TARGET", target)
    monkeypatch.setenv("MPEWALD_BATCH_SERIAL", one_stream)
    frames = _frames(FRAMES)
    desc, x, qoff, moff = _pack(frames)
    plan = _batch_plan(frames)
    print(f"[batch schedule] fwd_xcd={fwd_xcd} target={target} one_stream={one_stream}", flush=True)
    out = plan.batch(desc, *x)
    torch.cuda.synchronize()
    monkeypatch.delenv("MPEWALD_FWD_XCD")
    monkeypatch.delenv("MPEWALD_BATCH_TARGET")
    monkeypatch.delenv("MPEWALD_BATCH_SERIAL")
    for i, f in enumerate(frames):
        got = _per_frame(frames, out, qoff, moff, i)
        single = H.gpu_outputs(f)
        errs = H.compare(got, single, H.FWD_KEYS + H.BWD_KEYS)
        assert max(errs.values()) <= 1e-12, (i, errs)


def test_batch_frame_order_irrelevant():
    frames = _frames(FRAMES[:4])
    desc, x, qoff, moff = _pack(frames)
    out = _batch_plan(frames).batch(desc, *x)
    order = [2, 0, 3, 1]
    desc2, x2, qoff2, moff2 = _pack(frames, order)
    out2 = _batch_plan(frames).batch(desc2, *x2)
    torch.cuda.synchronize()
    for j, i in enumerate(order):
        a = _per_frame(frames, out, qoff, moff, i)
        b = _per_frame(frames, out2, qoff2, moff2, j)
        errs = H.compare(b, a, H.FWD_KEYS + H.BWD_KEYS)
        assert max(errs.values()) <= 1e-12, (i, errs)


def test_graph_replays_follow_inplace_input_changes():
    frames = _frames(FRAMES[:3])
    desc, x, qoff, moff = _pack(frames)
    plan = _batch_plan(frames)
    out = plan.batch(desc, *x)
    scales = [1.0, 2.0, -0.5, 1.0]
    q0 = x[5].clone()
    for sc in scales:
        x[5].copy_(q0 * sc)           # eager work between replays, same pointers
        plan.batch(desc, *x, out=out)  # replay
        torch.cuda.synchronize()
        for i, f in enumerate(frames):
            f2 = wl.System(**{**f.__dict__, "q": f.q * sc})
            got = _per_frame(frames, out, qoff, moff, i)
            single = H.gpu_outputs(f2)
            errs = H.compare(got, single, H.FWD_KEYS + H.BWD_KEYS)
            assert max(errs.values()) <= 1e-12, (sc, i, errs)


def test_forward_only_mode():
    frames = _frames(FRAMES[:2])
    desc, x, qoff, moff = _pack(frames)
    out = _batch_plan(frames).batch(desc, *x, with_grad=False)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        single = H.gpu_outputs(f, backward=False)
        o = {k: v.cpu().numpy() for k, v in out.items()}
        got = dict(energy=o["energy"][i], phi=o["phi"][qoff[i]:qoff[i + 1]],
                   efield=o["efield"][qoff[i]:qoff[i + 1]], efgrad=o["efgrad"][qoff[i]:qoff[i + 1]])
        assert max(H.compare(got, single, H.FWD_KEYS).values()) <= 1e-12


def test_capacity_errors():
    frames = _frames(FRAMES[:3])
    desc, x, qoff, moff = _pack(frames)
    plan = _batch_plan(frames[:2], max_frames=2)
    with pytest.raises(EwaldError) as ei:
        plan.batch(desc, *x)
    assert ei.value.status == EWALD_ERR_CAPACITY
    small = Plan(EwaldConfig(box=tuple(frames[0].box), alpha=0.3, rcut=8.0, kmax=8, max_qm=3, max_mm=100))
    d = H.to_dev(frames[0])
    with pytest.raises(EwaldError) as ei:
        small.forward(d["qm_pos"], d["Q"], d["mu"], d["theta"], d["mm_pos"], d["mm_q"])
    assert ei.value.status == EWALD_ERR_CAPACITY
