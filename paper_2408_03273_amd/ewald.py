"""PyTorch front-end of the HIP multipolar Ewald library.

PyTorch provides device memory and the current stream; every arithmetic step
runs in the library's kernels.  Tensors are float64, contiguous, on the
plan's device:

  qm_pos (Nq,3), Q (Nq,), mu (Nq,3), theta (Nq,6) raw second moments
  (xx,xy,xz,yy,yz,zz), mm_pos (Nm,3), mm_q (Nm,).

Outputs of the forward pass: energy (scalar), phi (Nq,), efield (Nq,3) = -grad
phi, efgrad (Nq,6) = -grad grad phi, where phi is the Ewald potential of the
MM charges at the QM sites (paper: periodic multipole energy; SI, multipolar
Ewald).  The energy includes the QM-QM image terms when the plan has
qmqm=True.  :class:`EwaldFunction` is the autograd adjoint: gradients with
respect to all six inputs (dE/d(moments) is the Fock-coupling potential of the
paper; minus the position gradients are the forces).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import EwaldError, check


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _req(t, shape, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, the plan is on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


@dataclass
class EwaldConfig:
    box: tuple
    alpha: float
    rcut: float
    kmax: tuple
    max_qm: int
    max_mm: int
    max_frames: int = 1
    qmqm: bool = True
    precision: str = "fp64"   # or "fp32_real", "fp32_recip" (reciprocal hot loops), "fp32_all"
    plain: bool = False       # unoptimised reference GPU path for the forward pass
    profile: object = False   # True: bracket every launch with HIP events; "hot": only the two hot loops
    cell_list: bool = True    # real space over cells of edge >= rcut when the box has >= 3 per axis
    background: bool = True   # uniform neutralising background of charged subsystems
    deterministic: bool = False  # fixed-order cross-block sums: bitwise reproducible outputs


@dataclass
class Region:
    """Region-I / region-II split (paper: periodic QM/MM multipole energy and
    the Gaussian-charge correction): region I is the sphere of radius r_region
    around the mean QM position; mm_kappa (Nm,) float64 on the plan's device
    gives Gaussian exponents (<= 0: point charge), r_gauss the pair cutoff of
    the Gaussian correction."""
    r_region: float
    r_gauss: float = 0.0
    mm_kappa: object = None


def suggest_params(box, rcut: float, tol: float):
    """(alpha, (mx, my, mz)) for a target truncation accuracy tol at this
    real-space cutoff (host-side estimate of the library; no GPU needed)."""
    lib = _lib.load()
    b = (ctypes.c_double * 3)(*[float(x) for x in box])
    alpha = ctypes.c_double()
    km = (ctypes.c_int * 3)()
    check(lib.ewald_suggest_params(b, float(rcut), float(tol), ctypes.byref(alpha), km))
    return alpha.value, tuple(km)


class Plan:
    """Owns a library plan (workspace on one device)."""

    def __init__(self, cfg: EwaldConfig, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU; none is visible")
        self.lib = _lib.load()
        self.cfg = cfg
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        p = _lib.EwaldParams()
        p.box[:] = [float(b) for b in cfg.box]
        p.alpha = float(cfg.alpha)
        p.rcut = float(cfg.rcut)
        km = (int(cfg.kmax),) * 3 if isinstance(cfg.kmax, int) else tuple(int(k) for k in cfg.kmax)
        p.kmax[:] = km
        p.precision = {"fp64": _lib.EWALD_FP64, "fp32_real": _lib.EWALD_FP32_REAL,
                       "fp32_recip": _lib.EWALD_FP32_RECIP,
                       "fp32_all": _lib.EWALD_FP32_REAL | _lib.EWALD_FP32_RECIP}[cfg.precision]
        p.flags = ((_lib.EWALD_QMQM if cfg.qmqm else 0) | (_lib.EWALD_PLAIN if cfg.plain else 0)
                   | (_lib.EWALD_PROFILE_HOT if cfg.profile == "hot" else _lib.EWALD_PROFILE if cfg.profile else 0)
                   | (_lib.EWALD_CELL_LIST if cfg.cell_list else 0)
                   | (0 if cfg.background else _lib.EWALD_NO_BACKGROUND)
                   | (_lib.EWALD_DETERMINISTIC if cfg.deterministic else 0))
        p.max_qm, p.max_mm, p.max_frames = int(cfg.max_qm), int(cfg.max_mm), int(cfg.max_frames)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self.lib.ewald_setup(ctypes.byref(p), ctypes.byref(h)))
        self.handle = h
        self.kmax = km

    def close(self):
        if getattr(self, "handle", None):
            self.lib.ewald_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def describe(self) -> str:
        return self.lib.ewald_plan_describe(self.handle).decode()

    def profile_report(self) -> dict:
        """Per-kernel launch counts and summed durations since the last report."""
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        check(self.lib.ewald_profile_report(self.handle, buf, len(buf)))
        return json.loads(buf.value.decode())

    def set_box(self, box):
        arr = (ctypes.c_double * 3)(*[float(b) for b in box])
        check(self.lib.ewald_set_box(self.handle, arr))

    def ctx_bytes(self, nq: int, nm: int) -> int:
        return int(self.lib.ewald_ctx_bytes(self.handle, nq, nm))

    def autotune(self, n_mm: int, cache_path: str | None = None):
        with torch.cuda.device(self.device):
            check(self.lib.ewald_autotune(self.handle, int(n_mm), cache_path.encode() if cache_path else None))

    # ------------------------------------------------------------------ raw calls
    def forward(self, qm_pos, Q, mu, theta, mm_pos, mm_q, want_ctx=False):
        dev = self.device
        nq, nm = int(Q.shape[0]), int(mm_q.shape[0])
        qm_pos = _req(qm_pos, (nq, 3), "qm_pos", dev)
        Q = _req(Q, (nq,), "Q", dev)
        mu = _req(mu, (nq, 3), "mu", dev)
        theta = _req(theta, (nq, 6), "theta", dev)
        mm_pos = _req(mm_pos, (nm, 3), "mm_pos", dev)
        mm_q = _req(mm_q, (nm,), "mm_q", dev)
        f64 = dict(dtype=torch.float64, device=dev)
        energy = torch.empty((), **f64)
        phi = torch.empty((nq,), **f64)
        efield = torch.empty((nq, 3), **f64)
        efgrad = torch.empty((nq, 6), **f64)
        ctx = torch.empty((self.ctx_bytes(nq, nm),), dtype=torch.uint8, device=dev) if want_ctx else None
        with torch.cuda.device(dev):
            check(self.lib.ewald_forward(self.handle, nq, _ptr(qm_pos), _ptr(Q), _ptr(mu), _ptr(theta), nm,
                                         _ptr(mm_pos), _ptr(mm_q), _ptr(energy), _ptr(phi), _ptr(efield),
                                         _ptr(efgrad), _ptr(ctx), _stream_ptr(dev)))
        return energy, phi, efield, efgrad, ctx

    def backward(self, ctx, qm_pos, Q, mu, theta, mm_pos, mm_q, gE=None, g_phi=None, g_efield=None, g_efgrad=None,
                 want_g_mm_q=True):
        dev = self.device
        nq, nm = int(Q.shape[0]), int(mm_q.shape[0])
        f64 = dict(dtype=torch.float64, device=dev)
        g_qm = torch.empty((nq, 3), **f64)
        g_Q = torch.empty((nq,), **f64)
        g_mu = torch.empty((nq, 3), **f64)
        g_th = torch.empty((nq, 6), **f64)
        g_mm = torch.empty((nm, 3), **f64)
        g_q = torch.empty((nm,), **f64) if want_g_mm_q else None
        gE_t = None if gE is None else _req(gE.reshape(()), (), "gE", dev)
        g_phi = None if g_phi is None else _req(g_phi, (nq,), "g_phi", dev)
        g_efield = None if g_efield is None else _req(g_efield, (nq, 3), "g_efield", dev)
        g_efgrad = None if g_efgrad is None else _req(g_efgrad, (nq, 6), "g_efgrad", dev)
        with torch.cuda.device(dev):
            check(self.lib.ewald_backward(self.handle, _ptr(ctx), nq, _ptr(qm_pos), _ptr(Q), _ptr(mu), _ptr(theta),
                                          nm, _ptr(mm_pos), _ptr(mm_q), _ptr(gE_t), _ptr(g_phi), _ptr(g_efield),
                                          _ptr(g_efgrad), _ptr(g_qm), _ptr(g_Q), _ptr(g_mu), _ptr(g_th),
                                          _ptr(g_mm), _ptr(g_q), _stream_ptr(dev)))
        return g_qm, g_Q, g_mu, g_th, g_mm, g_q

    def update_moments(self, ctx, qm_pos, Q, mu, theta, n_mm):
        """Energy and dE/d(Q, mu, theta) for new QM moments at the geometry of the
        forward call that filled ctx (self-consistent-field iterations): the
        stored MM field is reused, only the QM-QM image terms are recomputed."""
        dev = self.device
        nq = int(Q.shape[0])
        f64 = dict(dtype=torch.float64, device=dev)
        qm_pos = _req(qm_pos, (nq, 3), "qm_pos", dev)
        Q = _req(Q, (nq,), "Q", dev)
        mu = _req(mu, (nq, 3), "mu", dev)
        theta = _req(theta, (nq, 6), "theta", dev)
        energy = torch.empty((), **f64)
        g_Q = torch.empty((nq,), **f64)
        g_mu = torch.empty((nq, 3), **f64)
        g_th = torch.empty((nq, 6), **f64)
        with torch.cuda.device(dev):
            check(self.lib.ewald_moments_update(self.handle, _ptr(ctx), nq, _ptr(qm_pos), _ptr(Q), _ptr(mu),
                                                _ptr(theta), int(n_mm), _ptr(energy), _ptr(g_Q), _ptr(g_mu),
                                                _ptr(g_th), _stream_ptr(dev)))
        return energy, g_Q, g_mu, g_th

    # ------------------------------------------------------------------ region I / region II
    def _region_args(self, region, qm_pos, Q, mu, theta, mm_pos, mm_q):
        dev = self.device
        nq, nm = int(Q.shape[0]), int(mm_q.shape[0])
        kap = region.mm_kappa
        if kap is not None:
            kap = _req(kap, (nm,), "mm_kappa", dev)
        return (nq, _ptr(_req(qm_pos, (nq, 3), "qm_pos", dev)), _ptr(_req(Q, (nq,), "Q", dev)),
                _ptr(_req(mu, (nq, 3), "mu", dev)), _ptr(_req(theta, (nq, 6), "theta", dev)), nm,
                _ptr(_req(mm_pos, (nm, 3), "mm_pos", dev)), _ptr(_req(mm_q, (nm,), "mm_q", dev)), _ptr(kap),
                float(region.r_region), float(region.r_gauss))

    def region_forward(self, region, qm_pos, Q, mu, theta, mm_pos, mm_q, energy, phi=None, efield=None,
                       efgrad=None):
        """Add the region-I subtraction and the Gaussian-charge correction
        (:class:`Region`) to energy, phi, efield, efgrad in place."""
        args = self._region_args(region, qm_pos, Q, mu, theta, mm_pos, mm_q)
        with torch.cuda.device(self.device):
            check(self.lib.ewald_region_forward(self.handle, *args, _ptr(energy), _ptr(phi), _ptr(efield),
                                                _ptr(efgrad), _stream_ptr(self.device)))

    def region_backward(self, region, qm_pos, Q, mu, theta, mm_pos, mm_q, grads, gE=None, g_phi=None, g_efield=None,
                        g_efgrad=None):
        """Add the gradients of the region terms to grads = (g_qm, g_Q, g_mu,
        g_theta, g_mm, g_q) in place (g_q may be None)."""
        args = self._region_args(region, qm_pos, Q, mu, theta, mm_pos, mm_q)
        g_qm, g_Q, g_mu, g_th, g_mm, g_q = grads
        with torch.cuda.device(self.device):
            check(self.lib.ewald_region_backward(self.handle, *args, _ptr(gE), _ptr(g_phi), _ptr(g_efield),
                                                 _ptr(g_efgrad), _ptr(g_qm), _ptr(g_Q), _ptr(g_mu), _ptr(g_th),
                                                 _ptr(g_mm), _ptr(g_q), _stream_ptr(self.device)))

    def octupole_error(self, qm_pos, omega, mm_pos, mm_q, r_first: float, r_step: float, n_r: int, r_outer: float,
                       eps: float):
        """Charge-octupole error estimate of region II for R_cut = r_first +
        k r_step (k < n_r) and the R_cut the search picks (-1: none); omega
        (Nq,10) raw third moments xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz,
        zzz.  Returns (err (n_r,), r_cut ()) as device tensors."""
        dev = self.device
        nq, nm = int(qm_pos.shape[0]), int(mm_q.shape[0])
        qm_pos = _req(qm_pos, (nq, 3), "qm_pos", dev)
        omega = _req(omega, (nq, 10), "omega", dev)
        mm_pos = _req(mm_pos, (nm, 3), "mm_pos", dev)
        mm_q = _req(mm_q, (nm,), "mm_q", dev)
        f64 = dict(dtype=torch.float64, device=dev)
        err = torch.empty((int(n_r),), **f64)
        r_cut = torch.empty((), **f64)
        with torch.cuda.device(dev):
            check(self.lib.ewald_octupole_error(self.handle, nq, _ptr(qm_pos), _ptr(omega), nm, _ptr(mm_pos),
                                                _ptr(mm_q), int(n_r), float(r_first), float(r_step), float(r_outer),
                                                float(eps), _ptr(err), _ptr(r_cut), _stream_ptr(dev)))
        return err, r_cut

    def batch(self, frames, qm_pos, Q, mu, theta, mm_pos, mm_q, with_grad=True, out=None):
        """frames: list of dicts with box, n_qm, n_mm, qm_offset, mm_offset over packed arrays.

        Pass the dict returned by a previous call as `out` to reuse the output
        tensors; with unchanged frames, inputs and outputs the library replays
        its captured HIP graph instead of recapturing."""
        dev = self.device
        nf = len(frames)
        arr = (_lib.EwaldFrame * nf)()
        for i, fr in enumerate(frames):
            arr[i].box[:] = [float(b) for b in fr["box"]]
            arr[i].n_qm, arr[i].n_mm = int(fr["n_qm"]), int(fr["n_mm"])
            arr[i].qm_offset, arr[i].mm_offset = int(fr["qm_offset"]), int(fr["mm_offset"])
        nq, nm = int(Q.shape[0]), int(mm_q.shape[0])
        qm_pos = _req(qm_pos, (nq, 3), "qm_pos", dev)
        Q = _req(Q, (nq,), "Q", dev)
        mu = _req(mu, (nq, 3), "mu", dev)
        theta = _req(theta, (nq, 6), "theta", dev)
        mm_pos = _req(mm_pos, (nm, 3), "mm_pos", dev)
        mm_q = _req(mm_q, (nm,), "mm_q", dev)
        if out is None:
            f64 = dict(dtype=torch.float64, device=dev)
            out = dict(energy=torch.empty((nf,), **f64), phi=torch.empty((nq,), **f64),
                       efield=torch.empty((nq, 3), **f64), efgrad=torch.empty((nq, 6), **f64))
            if with_grad:
                out.update(g_qm_pos=torch.empty((nq, 3), **f64), g_Q=torch.empty((nq,), **f64),
                           g_mu=torch.empty((nq, 3), **f64), g_theta=torch.empty((nq, 6), **f64),
                           g_mm_pos=torch.empty((nm, 3), **f64), g_mm_q=torch.empty((nm,), **f64))
        self.run_batch(arr, qm_pos, Q, mu, theta, mm_pos, mm_q, out, with_grad)
        return out

    def run_batch(self, arr, qm_pos, Q, mu, theta, mm_pos, mm_q, out, with_grad):
        dev = self.device
        g = out if with_grad else {}
        with torch.cuda.device(dev):
            check(self.lib.ewald_batch(self.handle, len(arr), arr, _ptr(qm_pos), _ptr(Q), _ptr(mu), _ptr(theta),
                                       _ptr(mm_pos), _ptr(mm_q),
                                       _lib.EWALD_FWD_BWD if with_grad else _lib.EWALD_FWD, _ptr(out["energy"]),
                                       _ptr(out["phi"]), _ptr(out["efield"]), _ptr(out["efgrad"]),
                                       _ptr(g.get("g_qm_pos")), _ptr(g.get("g_Q")), _ptr(g.get("g_mu")),
                                       _ptr(g.get("g_theta")), _ptr(g.get("g_mm_pos")), _ptr(g.get("g_mm_q")),
                                       _stream_ptr(dev)))


class EwaldFunction(torch.autograd.Function):
    """E, phi, efield, efgrad = EwaldFunction.apply(plan, qm_pos, Q, mu, theta, mm_pos, mm_q).

    The backward pass is the library's adjoint (once differentiable).  The
    forward call already evaluates the gradients of E (its adjoint kernel runs
    beside the forward kernel on a second stream) and keeps them with the MM
    structure factor and the MM field data in the saved context; a backward
    with upstream gradients only on E scales them, one with upstream gradients
    on phi/efield/efgrad re-runs the adjoint.  Phases e^{i k.r} are recomputed,
    never stored.
    """

    @staticmethod
    def forward(ctx, plan, qm_pos, Q, mu, theta, mm_pos, mm_q, region=None):
        energy, phi, efield, efgrad, cbuf = plan.forward(qm_pos, Q, mu, theta, mm_pos, mm_q, want_ctx=True)
        if region is not None:
            plan.region_forward(region, qm_pos, Q, mu, theta, mm_pos, mm_q, energy, phi, efield, efgrad)
        # unused outputs get no upstream gradient (None) instead of zeros, so the
        # library can take its energy-only adjoint
        ctx.set_materialize_grads(False)
        ctx.plan = plan
        ctx.region = region
        ctx.save_for_backward(qm_pos, Q, mu, theta, mm_pos, mm_q, cbuf)
        return energy, phi, efield, efgrad

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gE, g_phi, g_efield, g_efgrad):
        qm_pos, Q, mu, theta, mm_pos, mm_q, cbuf = ctx.saved_tensors
        plan = ctx.plan
        need = ctx.needs_input_grad
        gE = torch.zeros((), dtype=torch.float64, device=plan.device) if gE is None else gE.contiguous()
        g_qm, g_Q, g_mu, g_th, g_mm, g_q = plan.backward(
            cbuf, qm_pos.contiguous(), Q.contiguous(), mu.contiguous(), theta.contiguous(), mm_pos.contiguous(),
            mm_q.contiguous(), gE=gE, g_phi=None if g_phi is None else g_phi.contiguous(),
            g_efield=None if g_efield is None else g_efield.contiguous(),
            g_efgrad=None if g_efgrad is None else g_efgrad.contiguous(), want_g_mm_q=bool(need[6]))
        if ctx.region is not None:
            plan.region_backward(ctx.region, qm_pos.contiguous(), Q.contiguous(), mu.contiguous(),
                                 theta.contiguous(), mm_pos.contiguous(), mm_q.contiguous(),
                                 (g_qm, g_Q, g_mu, g_th, g_mm, g_q), gE=gE,
                                 g_phi=None if g_phi is None else g_phi.contiguous(),
                                 g_efield=None if g_efield is None else g_efield.contiguous(),
                                 g_efgrad=None if g_efgrad is None else g_efgrad.contiguous())
        return (None, g_qm if need[1] else None, g_Q if need[2] else None, g_mu if need[3] else None,
                g_th if need[4] else None, g_mm if need[5] else None, g_q if need[6] else None, None)


def ewald(plan: Plan, qm_pos, Q, mu, theta, mm_pos, mm_q, region: Region | None = None):
    """Differentiable forward pass: returns (energy, phi, efield, efgrad).
    With a :class:`Region` the outputs are the region-II quantities (the
    region-I subtraction and the Gaussian-charge correction added)."""
    return EwaldFunction.apply(plan, qm_pos, Q, mu, theta, mm_pos, mm_q, region)


__all__ = ["EwaldConfig", "Plan", "Region", "EwaldFunction", "ewald", "EwaldError"]
