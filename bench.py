"""Benchmark: multipolar-Ewald QM/MM forward+backward frames/s on one MI355X.

Workload (headline): 70x70x72 A box, 35,000 MM point charges (>= 1 A apart,
neutral, U(-0.9,0.9)), 40 QM sites with charge, dipole and quadrupole, alpha
0.22 /A, real cutoff 12 A, |n| <= 24 per axis, FP64.  One step = the
differentiable forward pass (energy, potential, field and field gradient at
the QM sites) plus the adjoint (gradients for every QM and MM input) through
torch.autograd; inputs are resident in HBM when timing starts.

Prints ONE JSON line.  Extra keys: per-kernel durations, the roofline of the
dominant kernel (achieved algorithmic FP64 rate against the 78.6 TFLOP/s
vector peak), the unoptimised plain forward path, a 64-frame batched run and
the CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz; FP64 matrix cores: the same
FP32_PEAK_TFLOPS = 157.3  # FP32 vector (packed)
HBM_PEAK_GBS = 8000.0
METRIC = "QM/MM Ewald fwd+bwd frames/s at 35k MM charges; % FP64 roofline vs plain path"
PROFILES = os.path.join(ROOT, "profiles")


def n_half_space(m):
    mx, my, mz = m
    return ((2 * mx + 1) * (2 * my + 1) * (2 * mz + 1) - 1) // 2


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "ewald_internal.h"):
        with open(os.path.join(ROOT, "paper_2408_03273_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, src_hash: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(PROFILES, "traffic_c3.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != src_hash:
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the GPU reaches its steady clock only after some tens of steps (measured:
    # the first 30 steps after 5 warm-up ones run ~10 % slower than later ones)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the plain-path and batched measurements")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiles instead of timing candidates")
    ap.add_argument("--f3-only", action="store_true",
                    help="only the rc ~ L measurement of the c3 frame (its JSON object), e.g. under a profiler")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the FP64 batches (64 c4 frames, 16 c5 replicas; their JSON objects), e.g. under a profiler")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one device-to-device copy of 256 MiB (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2408_03273_amd import workloads as wl
    from paper_2408_03273_amd.ewald import EwaldConfig, Plan, ewald

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.f3_only:
        print(json.dumps(_f3(dev)), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch_c4": _batch_variants(dev, 4, 64, (), 10)["fp64"],
                          "c5_batch": _batch_variants(dev, 5, 16, (), 5)["fp64"]}), flush=True)
        return
    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    s = wl.make_config(3)
    nh = n_half_space(s.kmax)
    import tempfile
    cache = os.path.join(tempfile.mkdtemp(prefix="mpewald_tune_"), "tune.jsonl")

    def make_plan(profile):
        p = Plan(EwaldConfig(box=tuple(s.box), alpha=s.alpha, rcut=s.rcut, kmax=s.kmax, max_qm=s.nq, max_mm=s.nm,
                             profile=profile))
        if not args.no_autotune:
            p.autotune(s.nm, cache)   # times candidate tilings once (untimed setup); later plans read the cache
        return p

    def tens(a, grad=True):
        return torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=grad)

    inputs = [tens(a) for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]

    def step(p):
        for t in inputs:
            t.grad = None
        E, phi, efield, efgrad = ewald(p, *inputs)
        E.backward()
        return E

    def timed_steps(p, nsteps):
        for _ in range(args.warmup):
            step(p)
        torch.cuda.synchronize()
        if p.cfg.profile:
            p.profile_report()  # discard warm-up timings
        t0 = time.perf_counter()
        for _ in range(nsteps):
            E = step(p)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert np.isfinite(E.item())
        return (t1 - t0) * 1e3 / nsteps

    # headline: a plan without event brackets
    tplan = make_plan(False)
    ms = timed_steps(tplan, args.steps)
    tplan.close()
    # beside it, the same tiles with HIP events around the hot loops on their
    # own streams: the per-launch durations of the roofline come from these
    pplan = make_plan("hot")
    ms_hot = timed_steps(pplan, args.steps)
    hot_kern = pplan.profile_report()

    # roofline of the dominant hot kernel, from the events of the bracketed run.
    # Algorithmic flops per (k in the half space, MM atom): forward 4 (the
    # folded method's minimal count: one real multiply-add of Re/Im of
    # q e^{i(kx x + ky y)} with cos and with sin of p kz0 z per (column, |nz|)
    # covers both k = (kx, ky, +-p kz0)), adjoint 6 (the forces: the imaginary
    # part of the product with the QM structure factor and the k-weighted
    # accumulation).  Executed by the matrix-core kernels: 4 and 8 (the adjoint
    # also forms the potential, dE/dq, and the nz-weighted sums).
    per = {k: dict(count=v["count"], avg_us=1e3 * v["total_ms"] / max(v["count"], 1),
                   ms_per_step=v["total_ms"] / args.steps) for k, v in hot_kern.items()}
    flops = {"sfac_mm": 4.0 * nh * s.nm, "force_mm": 6.0 * nh * s.nm}
    executed = {"sfac_mm": 4.0 * nh * s.nm, "force_mm": 8.0 * nh * s.nm}
    hot = {k: per[k] for k in flops if k in per}
    dom = max(hot, key=lambda k: hot[k]["ms_per_step"])
    achieved = flops[dom] / (per[dom]["avg_us"] * 1e-6) / 1e12
    src_hash = kernel_source_hash()
    # the dominant kernel runs on the FP64 matrix cores when the plan uses the
    # matrix-core variants (the FP64 MFMA and VALU peaks are both 78.6 TFLOP/s)
    mfma = ("bwd=mfma" in pplan.describe()) if dom == "force_mm" else ("fwd=mfma" in pplan.describe())
    roof = dict(bound="mfma" if mfma else "alu", achieved=round(achieved, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / FP64_PEAK_TFLOPS, 4), traffic=traffic_from_profiles(dom, src_hash),
                kernel=dom, flops_per_launch=flops[dom], avg_launch_us=round(per[dom]["avg_us"], 2),
                executed_flops_per_launch=executed[dom],
                executed_frac=round(executed[dom] / (per[dom]["avg_us"] * 1e-6) / 1e12 / FP64_PEAK_TFLOPS, 4))
    # the same kernel launched alone: the autotuner's standalone timing of the
    # chosen candidate (HIP events around repeated launches on a synthetic frame
    # of the same size, before the timed region); inside the step the two hot
    # loops and the QM-side kernels share the GPU, so the in-step duration above
    # also holds the time the kernel's blocks wait for room
    iso = _isolated_us(cache, pplan.describe(), dom)
    roof["isolated_avg_us"] = iso
    roof["isolated_frac"] = None if iso is None else round(flops[dom] / (iso * 1e-6) / 1e12 / FP64_PEAK_TFLOPS, 4)
    # the same against the FP64 throughput this GPU reaches with the library's
    # probe kernels (back-to-back matrix-core / VALU chains)
    peaks = _fp64_peaks(dev)
    roof["measured_peak_tflops"] = peaks
    unit_peak = peaks.get("mfma_f64" if mfma else "valu_f64")
    roof["isolated_executed_frac_vs_measured"] = (None if iso is None or not unit_peak else
                                                  round(executed[dom] / (iso * 1e-6) / 1e12 / unit_peak, 4))
    hot_total_us = sum(per[k]["avg_us"] for k in hot)
    path_flops = 10.0 * nh * s.nm
    path_exec = 12.0 * nh * s.nm
    extra = dict(
        hot_path=dict(kernels={k: dict(avg_us=round(per[k]["avg_us"], 2),
                                       algorithmic_frac=round(flops[k] / (per[k]["avg_us"] * 1e-6) / 1e12
                                                              / FP64_PEAK_TFLOPS, 4),
                                       executed_frac=round(executed[k] / (per[k]["avg_us"] * 1e-6) / 1e12
                                                           / FP64_PEAK_TFLOPS, 4)) for k in sorted(hot)},
                      flops_per_step=path_flops, executed_flops_per_step=path_exec, kernel_us=round(hot_total_us, 2),
                      ms_per_step_bracketed=round(ms_hot, 4),
                      step_frac_of_fp64_peak=round(path_flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                      step_executed_frac_of_fp64_peak=round(path_exec / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)),
        flop_model="per (k in the half space, MM atom): forward 4 (folded minimal count), adjoint 6 (forces); "
                   "executed 4 + 8",
        kernel_source_hash=src_hash, plan=pplan.describe())

    # every launch timed separately (events perturb the step, so not in the timed region)
    fplan = make_plan(True)
    for _ in range(3):
        step(fplan)
    torch.cuda.synchronize()
    fplan.profile_report()
    nprof = 5
    for _ in range(nprof):
        step(fplan)
    torch.cuda.synchronize()
    extra["kernels"] = {k: dict(avg_us=round(1e3 * v["total_ms"] / max(v["count"], 1), 2),
                                per_step=round(v["count"] / nprof, 2)) for k, v in fplan.profile_report().items()}
    fplan.close()

    if not args.no_extras:
        extra["scf_moments_update"] = _scf_update(make_plan(False), inputs, s, ms)
        extra["plain_path"] = _plain_path(s, dev, nh)
        # the optimised step (forward + adjoint) against the plain forward-only path
        extra["vs_plain_path"] = round(extra["plain_path"]["ms_per_frame_fwd"] / ms, 2)
        extra["batch_c4"] = _batch_c4(dev)
        extra["region_c3"] = _region_c3(make_plan(True), inputs, s)
        extra["fp32_recip"] = _fp32_recip(make_plan(False), s, inputs, cache, args.no_autotune)
        extra["per_config"] = _per_config(dev, args.no_autotune)
        extra["per_config"]["f3_c3_rc_near_L"] = _f3(dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(s)

    line = {
        "metric": METRIC, "value": round(1e3 / ms, 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c3: box 70x70x72 A, 35000 MM charges, 40 QM multipole sites, alpha 0.22, rcut 12 A, "
                               "|n|<=24, fwd+bwd via autograd, FP64",
                   "n_mm": s.nm, "n_qm": s.nq, "kmax": list(s.kmax), "n_kvec_half_space": nh,
                   "alpha": s.alpha, "rcut": s.rcut, "box": list(map(float, s.box)), "input_sha256": s.sha256()[:16]},
        "roofline": roof, "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


def _scf_update(plan, inputs, s, step_ms, calls=20):
    """Moments-only update at fixed geometry (one SCF iteration): energy and
    dE/d(moments) for new moments, reusing the MM field of one forward call."""
    import torch
    x = [t.detach() for t in inputs]
    _, _, _, _, ctx = plan.forward(*x, want_ctx=True)
    Q2, mu2, th2 = x[1] * 0.9, x[2] * 1.1, x[3] * 0.95
    plan.update_moments(ctx, x[0], Q2, mu2, th2, s.nm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        plan.update_moments(ctx, x[0], Q2, mu2, th2, s.nm)
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) * 1e6 / calls
    plan.close()
    return dict(us_per_call=round(us, 1), vs_full_step=round(step_ms * 1e3 / us, 1))


def _fp64_peaks(dev, blocks=2048):
    """FP64 TFLOP/s reached by the library's probe kernels on this GPU: v_mfma_f64
    16x16x4 in four independent chains per wave, and VALU FMAs in eight chains
    per lane (mean of five launches of ~1-2 ms, HIP events on the stream)."""
    import ctypes

    import torch

    from paper_2408_03273_amd import _lib
    lib = _lib.load()
    out = torch.empty(4 * blocks, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for kind, name, iters in ((0, "mfma_f64", 2000), (1, "valu_f64", 16000)):
        fl = ctypes.c_double(0.0)

        def run():
            _lib.check(lib.ewald_fp64_probe(kind, blocks, iters, ctypes.c_void_p(out.data_ptr()), ctypes.byref(fl),
                                            ctypes.c_void_p(stream.cuda_stream)))

        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        res[name] = round(fl.value / (ms * 1e-3) / 1e12, 2)
    return res


def _isolated_us(cache, describe, kernel):
    """Standalone launch time (us) of the plan's hot-loop candidate from the autotune cache, or None."""
    import re
    try:
        lines = open(cache).read().strip().splitlines()
    except OSError:
        return None
    if not lines:
        return None
    times = json.loads(lines[-1]).get("times_us", {})
    if kernel == "force_mm":
        m = re.search(r"bwd=mfma-fold-eyl xcd=(\d)(?: kc=(\d+))?", describe)
        if not m:
            return None
        keys = [k for k in times if k.startswith("bwd6_") and k.endswith(f"_x{m.group(1)}")
                and (m.group(2) is None or k.startswith(f"bwd6_kc{m.group(2)}_"))]
    else:
        m = re.search(r"fwd=mfma-fold ct=(\d) nt=\d xcd=(\d) blocks~(\d+)", describe)
        if not m:
            return None
        keys = [f"fwd_mfma_ct{m.group(1)}_{m.group(3)}_x{m.group(2)}"]
    vals = [times[k] for k in keys if k in times]
    return round(min(vals), 2) if vals else None


def _per_config(dev, no_autotune, steps=5):
    """Every configuration against the algorithmic model (10 flops per (k, MM
    atom) forward + adjoint, 4 forward only): c1, c2 as single frames through
    autograd, c5 as one batched call of its 16 replicas (FP64 and the mixed-
    precision variants, with their deviation from FP64), and the plain forward
    path (one thread per k, sincos per term) on c1, c2, c3 and one c5 replica."""
    import numpy as np
    import torch

    from paper_2408_03273_amd import workloads as wl
    from paper_2408_03273_amd.ewald import EwaldConfig, Plan, ewald

    def timed(fn, n):
        for _ in range(max(3, n)):  # warm-up: as many untimed calls as timed ones
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    def frac(fl, ms):
        return round(fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)

    out = {}
    for cfg in (1, 2):
        s = wl.make_config(cfg)
        nh = n_half_space(s.kmax)
        plan = Plan(EwaldConfig(box=tuple(s.box), alpha=s.alpha, rcut=s.rcut, kmax=s.kmax, max_qm=s.nq, max_mm=s.nm))
        if not no_autotune:
            plan.autotune(s.nm)
        x = [torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True)
             for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]

        def step():
            for t in x:
                t.grad = None
            ewald(plan, *x)[0].backward()

        ms = timed(step, 4 * steps)
        # the same frame as a one-frame batch: the launch sequence replays as one HIP graph
        xd = [t.detach() for t in x]
        desc = [dict(box=s.box, n_qm=s.nq, n_mm=s.nm, qm_offset=0, mm_offset=0)]
        ob = plan.batch(desc, *xd)
        ms_g = timed(lambda: plan.batch(desc, *xd, out=ob), 4 * steps)
        out[f"c{cfg}"] = dict(n_mm=s.nm, n_kvec_half_space=nh, ms_per_frame_fwd_bwd=round(ms, 4),
                              frames_per_s=round(1e3 / ms, 1), frac_of_fp64_peak=frac(10.0 * nh * s.nm, ms),
                              graph_replay_ms=round(ms_g, 4), graph_replay_frac=frac(10.0 * nh * s.nm, ms_g))
        plan.close()
    # c5: 16 replicas of 100 000 MM charges, FP64 and the mixed-precision variants
    v = _batch_variants(dev, 5, 16, ("fp32_real", "fp32_recip", "fp32_all"), steps)
    out["c5_batch"] = v["fp64"]
    out["c5_batch"]["mixed_precision"] = {k: v[k] for k in ("fp32_real", "fp32_recip", "fp32_all")}
    plain = {}
    for cfg in (1, 2, 3, 5):
        s = wl.make_config(cfg)
        nh = n_half_space(s.kmax)
        plan = Plan(EwaldConfig(box=tuple(s.box), alpha=s.alpha, rcut=s.rcut, kmax=s.kmax, max_qm=s.nq, max_mm=s.nm,
                                plain=True))
        x = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]
        ms = timed(lambda: plan.forward(*x), 2 if cfg == 5 else steps)
        plain[f"c{cfg}"] = dict(ms_per_frame_fwd=round(ms, 3), frac_of_fp64_peak=frac(4.0 * nh * s.nm, ms))
        plan.close()
    out["plain_forward"] = plain
    return out


def _fp32_recip(plan64, s, inputs, cache, no_autotune, steps=100):
    """The same c3 step with the two reciprocal hot loops on FP32 matrix cores
    (mixed-precision variant); its deviation from the FP64 path is reported
    (normwise relative, per output)."""
    import torch

    from paper_2408_03273_amd.ewald import EwaldConfig, Plan, ewald

    def run(plan):
        x = [t.detach().clone().requires_grad_(True) for t in inputs]
        E, phi, ef, eg = ewald(plan, *x)
        E.backward()
        return [E.detach(), phi.detach(), ef.detach(), eg.detach()] + [t.grad for t in x]

    ref = run(plan64)
    plan64.close()
    plan = Plan(EwaldConfig(box=tuple(s.box), alpha=s.alpha, rcut=s.rcut, kmax=s.kmax, max_qm=s.nq, max_mm=s.nm,
                            precision="fp32_recip"))
    if not no_autotune:
        plan.autotune(s.nm, cache)
    got = run(plan)
    names = ("energy", "phi", "efield", "efgrad", "g_qm_pos", "g_Q", "g_mu", "g_theta", "g_mm_pos", "g_mm_q")
    err = {n: float((a - b).abs().max() / b.abs().max()) for n, a, b in zip(names, got, ref)}
    x = [t.detach().clone().requires_grad_(True) for t in inputs]
    for _ in range(steps):
        ewald(plan, *x)[0].backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for t in x:
            t.grad = None
        ewald(plan, *x)[0].backward()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    desc = plan.describe()
    plan.close()
    return dict(frames_per_s=round(1e3 / ms, 1), ms_per_step=round(ms, 4), plan=desc,
                rel_err_vs_fp64={k: float(f"{v:.2e}") for k, v in err.items()},
                max_rel_err=float(f"{max(err.values()):.2e}"), dtype="f32 matrix cores, f64 sums")


def _region_c3(plan, inputs, s, calls=20):
    """Region-II quantities on the c3 frame: the region-I subtraction (sphere
    of 16 A around the QM centre) and the Gaussian-charge correction (kappa =
    1/r_cov, pairs within 5 A), forward and adjoint; and the charge-octupole
    error estimate for 16 candidate radii 13..28 A (outer radius 35 A)."""
    import numpy as np
    import torch

    from paper_2408_03273_amd import workloads as wl
    from paper_2408_03273_amd.ewald import Region
    x = [t.detach() for t in inputs]
    dev = x[0].device
    reg = Region(16.0, 5.0, torch.tensor(wl.gaussian_exponents(3, s.nm), dtype=torch.float64, device=dev))
    E = torch.zeros((), dtype=torch.float64, device=dev)
    phi, ef, eg = (torch.zeros((s.nq,) + sh, dtype=torch.float64, device=dev) for sh in ((), (3,), (6,)))
    grads = tuple(torch.zeros_like(t) for t in (x[0], x[1], x[2], x[3], x[4], x[5]))
    omega = torch.tensor(np.random.default_rng(3).normal(0.0, 0.05, (s.nq, 10)), dtype=torch.float64, device=dev)

    def fwd_bwd():
        plan.region_forward(reg, *x, E, phi, ef, eg)
        plan.region_backward(reg, *x, grads)

    def octupole():
        plan.octupole_error(x[0], omega, x[4], x[5], 13.0, 1.0, 16, 35.0, 1e-4)

    out = {}
    for name, fn in (("fwd_bwd_wall_us", fwd_bwd), ("octupole_wall_us", octupole)):
        fn()
        torch.cuda.synchronize()
        plan.profile_report()
        t0 = time.perf_counter()
        for _ in range(calls):
            fn()
        torch.cuda.synchronize()
        out[name] = round((time.perf_counter() - t0) * 1e6 / calls, 1)
        # GPU time of each entry point's launch sequence (events around it on the stream)
        for k, v in plan.profile_report().items():
            out[k + "_gpu_us"] = round(1e3 * v["total_ms"] / max(v["count"], 1), 1)
    c = s.qm_pos.mean(0)
    d = s.mm_pos - c
    d -= s.box * np.rint(d / s.box)
    out.update(r_region=16.0, r_gauss=5.0, region_translates=int(np.sum(np.sum(d * d, 1) < 16.0 ** 2)),
               octupole_candidates=16)
    plan.close()
    return out


def _plain_path(s, dev, nh, steps=5):
    """Unoptimised forward path (one thread per k, sincos per (k, atom))."""
    import torch

    from paper_2408_03273_amd.ewald import EwaldConfig, Plan
    plan = Plan(EwaldConfig(box=tuple(s.box), alpha=s.alpha, rcut=s.rcut, kmax=s.kmax, max_qm=s.nq, max_mm=s.nm,
                            plain=True))
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    x = [t(a) for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]
    plan.forward(*x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward(*x)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    fl = 4.0 * nh * s.nm
    plan.close()
    return dict(ms_per_frame_fwd=round(ms, 3), frames_per_s_fwd=round(1e3 / ms, 2),
                frac_of_fp64_peak=round(fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4))


def _rel_errs(got, ref):
    """Normwise relative deviation per output array: max|a - b| / max|b|."""
    return {k: float((got[k] - ref[k]).abs().max() / ref[k].abs().max()) for k in ref if ref[k].abs().max() > 0}


def _batch_variants(dev, cfg, nframes, variants, steps):
    """One batch of frames of configuration cfg through graph-replayed batch
    calls, FP64 and the given precision variants (each against the FP64
    outputs of the same call: normwise relative deviation per output)."""
    import numpy as np
    import torch

    from paper_2408_03273_amd import workloads as wl
    from paper_2408_03273_amd.ewald import EwaldConfig, Plan
    frames = [wl.make_config(cfg, f) for f in range(nframes)]
    qoff = np.cumsum([0] + [f.nq for f in frames])
    moff = np.cumsum([0] + [f.nm for f in frames])
    desc = [dict(box=f.box, n_qm=f.nq, n_mm=f.nm, qm_offset=int(qoff[i]), mm_offset=int(moff[i]))
            for i, f in enumerate(frames)]
    cat = lambda k: torch.tensor(np.concatenate([getattr(f, k) for f in frames]), dtype=torch.float64,  # noqa: E731
                                 device=dev)
    x = [cat("qm_pos"), cat("Q"), cat("mu"), cat("theta"), cat("mm_pos"), cat("q")]
    f0 = frames[0]
    nh = n_half_space(f0.kmax)
    fl = 10.0 * nh * float(moff[-1])
    out, ref = {}, None
    for prec in ("fp64",) + tuple(variants):
        plan = Plan(EwaldConfig(box=tuple(f0.box), alpha=f0.alpha, rcut=f0.rcut, kmax=f0.kmax, max_qm=int(qoff[-1]),
                                max_mm=int(moff[-1]), max_frames=nframes, precision=prec))
        if cfg == 5 or prec == "fp32_recip" or prec == "fp32_all":
            plan.autotune(f0.nm)
        o = plan.batch(desc, *x)
        for _ in range(steps):  # warm-up (steady clocks)
            plan.batch(desc, *x, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.batch(desc, *x, out=o)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        r = dict(frames=nframes, total_mm=int(moff[-1]), ms_per_batch=round(ms, 3),
                 frames_per_s=round(nframes * 1e3 / ms, 1),
                 frac_of_fp64_peak=round(fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4), plan=plan.describe())
        if ref is None:
            ref = {k: v.clone() for k, v in o.items()}
        else:
            err = _rel_errs(o, ref)
            r["rel_err_vs_fp64"] = {k: float(f"{v:.2e}") for k, v in err.items()}
            r["max_rel_err"] = float(f"{max(err.values()):.2e}")
        out[prec] = r
        plan.close()
    return out


def real_flops_from_profiles(precision: str, src_hash: str):
    """Executed FP64 and FP32 flops per real-space pair (both sides of the
    pair) from the committed counter summary of the lattice-image kernel, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(PROFILES, "real_img_f3.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != src_hash:
        return None
    return d.get("per_pair", {}).get(precision)


def _f3(dev, steps=20):
    """The paper's regime: the c3 frame with a real-space cutoff of 0.95 of the
    smallest box edge and alpha, kmax from the parameter suggestion at 1e-8
    (real space sums up to 8 lattice images per pair and dominates; the k-set
    is small).  FP64 and FP32 real space (FP64 accumulation): the autograd
    step, the same frame as a graph-replayed one-frame batch, the real-space
    launch alone (HIP events), pairs within the cutoff per second, and the
    real-space kernel against the VALU peak with its executed flops per pair
    (hardware counters: FP64 against 78.6, FP32 against 157.3 TFLOP/s)."""
    import numpy as np
    import torch

    from paper_2408_03273_amd import workloads as wl
    from paper_2408_03273_amd.ewald import EwaldConfig, Plan, ewald, suggest_params

    s = wl.make_config(3)
    rc = 0.95 * float(np.min(s.box))
    alpha, kmax = suggest_params(s.box, rc, 1e-8)
    # pairs (site, atom, lattice image) within the cutoff
    d = s.qm_pos[:, None, :] - s.mm_pos[None, :, :]
    d -= s.box * np.round(d / s.box)
    pairs = 0
    for n in np.ndindex(3, 3, 3):
        e = d + (np.array(n) - 1) * s.box
        pairs += int(((e * e).sum(-1) < rc * rc).sum())
    del d
    src_hash = kernel_source_hash()
    out = dict(workload=f"c3 frame, rc = 0.95 L = {rc:.1f} A, alpha {alpha:.4f}, kmax {list(kmax)} "
                        "(parameters for 1e-8), fwd+bwd via autograd",
               n_mm=s.nm, n_qm=s.nq, rcut=rc, alpha=round(alpha, 6), kmax=list(kmax),
               n_kvec_half_space=n_half_space(kmax), real_space_pairs=pairs)
    x = [torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True)
         for a in (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)]
    xd = [t.detach() for t in x]
    desc = [dict(box=s.box, n_qm=s.nq, n_mm=s.nm, qm_offset=0, mm_offset=0)]
    ref = None
    for prec in ("fp64", "fp32_real"):
        r = {}
        for prof in (False, True):
            plan = Plan(EwaldConfig(box=tuple(s.box), alpha=alpha, rcut=rc, kmax=kmax, max_qm=s.nq, max_mm=s.nm,
                                    precision=prec, profile=prof))

            def step():
                for t in x:
                    t.grad = None
                ewald(plan, *x)[0].backward()

            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            if prof:
                plan.profile_report()
                for _ in range(steps):
                    step()
                torch.cuda.synchronize()
                k = plan.profile_report()["real_qm"]
                r["real_space_us"] = round(1e3 * k["total_ms"] / k["count"], 2)
            else:
                t0 = time.perf_counter()
                for _ in range(steps):
                    step()
                torch.cuda.synchronize()
                r["ms_per_frame_fwd_bwd"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
                ob = plan.batch(desc, *xd)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    plan.batch(desc, *xd, out=ob)
                torch.cuda.synchronize()
                r["graph_replay_ms"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
                if ref is None:
                    ref = {k: v.clone() for k, v in ob.items()}
                else:
                    err = _rel_errs(ob, ref)
                    r["max_rel_err_vs_fp64"] = float(f"{max(err.values()):.2e}")
            plan.close()
        t = r["real_space_us"] * 1e-6
        r["pairs_per_s"] = float(f"{pairs / t:.4g}")
        fl = real_flops_from_profiles(prec, src_hash)
        if fl is not None:
            f64, f32 = fl["fp64"] * pairs, fl["fp32"] * pairs
            # share of the launch the VALU would need at peak for these flops
            frac = (f64 / FP64_PEAK_TFLOPS + f32 / FP32_PEAK_TFLOPS) / 1e12 / t
            r["roofline"] = dict(bound="alu", kernel="real space, lattice images (k_real_img)",
                                 executed_fp64_flops_per_pair=fl["fp64"], executed_fp32_flops_per_pair=fl["fp32"],
                                 achieved_fp64_tflops=round(f64 / t / 1e12, 3),
                                 achieved_fp32_tflops=round(f32 / t / 1e12, 3),
                                 peak_fp64_tflops=FP64_PEAK_TFLOPS, peak_fp32_tflops=FP32_PEAK_TFLOPS,
                                 frac=round(frac, 4))
        else:
            r["roofline"] = None
        out[prec] = r
    return out


def _batch_c4(dev, steps=10):
    """64 independent frames of uneven size through one graph-replayed batch
    call, FP64 and with the real space in FP32 (FP64 accumulation)."""
    v = _batch_variants(dev, 4, 64, ("fp32_real",), steps)
    res = v["fp64"]
    res["fp32_real"] = v["fp32_real"]
    return res


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(s):
    """The FP64 CPU oracle, as it stands, built for this host (gcc -O3
    -march=native -fopenmp, in a temporary directory) and timed on one full c3
    frame (forward and every gradient) with all OpenMP threads, and on a
    sample of the frame (its first 5000 MM charges, scaled to a whole frame by
    the MM count, which the oracle's time is linear in) with one thread."""
    import tempfile

    import numpy as np

    from oracle import oracle as orc
    lib = os.path.join(tempfile.mkdtemp(prefix="mpewald_oracle_"), "libewald_oracle_native.so")
    orc.build(out=lib, extra_flags=("-O3", "-march=native"))
    # the host share this process may use (the OpenMP setting where there is one)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    orc.set_num_threads(threads, lib_path=lib)
    t0 = time.perf_counter()
    r = orc.oracle_ewald(s.box, s.alpha, s.rcut, s.kmax, s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q, lib_path=lib)
    dt = time.perf_counter() - t0
    assert np.isfinite(r.E)
    n1 = 5000
    orc.set_num_threads(1, lib_path=lib)
    t0 = time.perf_counter()
    r1 = orc.oracle_ewald(s.box, s.alpha, s.rcut, s.kmax, s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos[:n1], s.q[:n1],
                          lib_path=lib)
    dt1 = time.perf_counter() - t0
    assert np.isfinite(r1.E)
    frame1 = dt1 * s.nm / n1
    return dict(value=round(1.0 / dt, 5), unit="frames/s", cores=threads, kind="oracle",
                sample="one full c3 frame (35000 MM, 40 QM, |n|<=24): energy, fields and every gradient",
                seconds=round(dt, 2), cpu_model=_cpu_model(), build="gcc -O3 -march=native -fopenmp",
                single_thread=dict(value=round(1.0 / frame1, 5), unit="frames/s", cores=1,
                                   sample=f"the c3 frame with its first {n1} MM charges, "
                                          f"{dt1:.2f} s, scaled by {s.nm}/{n1}",
                                   seconds_per_frame=round(frame1, 2)))


if __name__ == "__main__":
    main()
