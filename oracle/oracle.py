"""Plain FP64 CPU oracle for the multipolar-Ewald QM/MM coupling (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It compiles ``ewald_oracle.c`` with gcc (no code shared
with the HIP library) and exposes :func:`oracle_ewald` (the Ewald sums) and
:func:`oracle_region` (the region-I subtraction and Gaussian-charge correction).

Conventions (paper: SI "Multipolar Ewald"; main text, periodic QM/MM energy):
  * positions in length units (Angstrom in the workloads), charges in e,
    Coulomb constant 1, so energies come out in e^2/Angstrom;
  * theta is the raw second moment, stored as (xx, xy, xz, yy, yz, zz);
  * phi, dphi, hphi are the MM-generated Ewald potential, its gradient and
    one half of its Hessian at each QM site;
  * g_* are derivatives of the total energy E = E_QMMM + E_QQ; g_theta is the
    derivative with respect to the six stored numbers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ewald_oracle.c")
_DEFAULT_LIB = os.path.join(_HERE, "libewald_oracle.so")
# MPEWALD_ORACLE_LIB names another build of the oracle (e.g. a sanitized one), used as it is
_LIB = os.environ.get("MPEWALD_ORACLE_LIB") or _DEFAULT_LIB

ENERGY_NAMES = ("total", "qmmm_sr", "qmmm_lr", "qmmm_bg", "qq_sr", "qq_lr", "qq_self", "qq_bg")


class _Params(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("alpha", ctypes.c_double),
        ("rcut", ctypes.c_double),
        ("kmax", ctypes.c_int * 3),
        ("qmqm", ctypes.c_int),
        ("background", ctypes.c_int),
    ]


def build(src: str = _SRC, out: str = _DEFAULT_LIB, extra_flags: tuple = ()) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, generic x86-64)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-fno-fast-math",
           "-ffp-contract=off", *extra_flags, "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib_cache: dict = {}


def load(path: str = _LIB) -> ctypes.CDLL:
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path) or (path == _DEFAULT_LIB and os.path.getmtime(path) < os.path.getmtime(_SRC)):
        if path != _DEFAULT_LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_ewald.restype = ctypes.c_int
    lib.oracle_ewald.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, dp, dp,
                                 dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int, ip, dp, dp]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    lib.oracle_region.restype = ctypes.c_int
    lib.oracle_octupole_error.restype = ctypes.c_int
    lib.oracle_octupole_error.argtypes = [dp, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_int, dp,
                                          ctypes.c_double, dp]
    lib.oracle_rcut_pick.restype = ctypes.c_double
    lib.oracle_rcut_pick.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double]
    lib.oracle_region.argtypes = [ctypes.POINTER(_RegionParams), ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, dp, dp,
                                  dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_long)]
    _lib_cache[path] = lib
    return lib


def num_threads() -> int:
    return int(load().oracle_num_threads())


def set_num_threads(n: int, lib_path: str | None = None) -> None:
    """OpenMP threads of later oracle calls (for timing)."""
    (load(lib_path) if lib_path else load()).oracle_set_num_threads(int(n))


@dataclass
class OracleResult:
    energy: dict
    phi: np.ndarray        # (nq,)
    dphi: np.ndarray       # (nq,3)   grad phi
    hphi: np.ndarray       # (nq,6)   1/2 grad grad phi
    g_qm_pos: np.ndarray   # (nq,3)   dE/dR_qm
    g_Q: np.ndarray        # (nq,)
    g_mu: np.ndarray       # (nq,3)
    g_theta: np.ndarray    # (nq,6)   w.r.t. stored numbers
    g_mm_pos: np.ndarray   # (nsel,3) dE/dR_mm
    g_mm_q: np.ndarray     # (nsel,)
    mm_sel: np.ndarray | None

    @property
    def E(self) -> float:
        return self.energy["total"]

    @property
    def efield(self) -> np.ndarray:
        return -self.dphi

    @property
    def efgrad(self) -> np.ndarray:
        """-grad grad phi in (xx,xy,xz,yy,yz,zz) order."""
        return -2.0 * self.hphi


def _c(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def oracle_ewald(box, alpha, rcut, kmax, qm_pos, Q, mu, theta, mm_pos, q, qmqm=True, mm_sel=None,
                 lib_path: str | None = None, background=True) -> OracleResult:
    """Evaluate the truncated Ewald sums for the given parameters.

    box: (3,) orthorhombic edges; kmax: int or (3,) per-axis |n| limit;
    qm_pos (nq,3), Q (nq,), mu (nq,3), theta (nq,6); mm_pos (nm,3), q (nm,).
    mm_sel: optional indices of MM atoms whose gradients are wanted.
    background: include the uniform neutralising background of charged
    subsystems (the paper is silent on it; on by default).
    """
    lib = load(lib_path) if lib_path else load()
    qm_pos = _c(qm_pos).reshape(-1, 3)
    nq = qm_pos.shape[0]
    Q = _c(Q, (nq,))
    mu = _c(mu, (nq, 3))
    theta = _c(theta, (nq, 6))
    mm_pos = _c(mm_pos).reshape(-1, 3)
    nm = mm_pos.shape[0]
    q = _c(q, (nm,))
    if np.isscalar(kmax):
        kmax = (int(kmax),) * 3
    p = _Params()
    p.box[:] = [float(b) for b in box]
    p.alpha = float(alpha)
    p.rcut = float(rcut)
    p.kmax[:] = [int(k) for k in kmax]
    p.qmqm = 1 if qmqm else 0
    p.background = 1 if background else 0
    if mm_sel is None:
        nsel = nm
        sel_arg = None
        sel_n = -1
    else:
        sel = np.ascontiguousarray(np.asarray(mm_sel, dtype=np.int32))
        if sel.size and (sel.min() < 0 or sel.max() >= nm):
            raise IndexError("mm_sel out of range")
        nsel = sel.size
        sel_arg = sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        sel_n = nsel
    energy = np.zeros(len(ENERGY_NAMES))
    phi = np.zeros(nq)
    dphi = np.zeros((nq, 3))
    hphi = np.zeros((nq, 6))
    gq = np.zeros((nq, 3))
    gQ = np.zeros(nq)
    gmu = np.zeros((nq, 3))
    gth = np.zeros((nq, 6))
    gm = np.zeros((max(nsel, 0), 3))
    gmq = np.zeros(max(nsel, 0))
    rc = lib.oracle_ewald(ctypes.byref(p), nq, _ptr(qm_pos), _ptr(Q), _ptr(mu), _ptr(theta), nm, _ptr(mm_pos),
                          _ptr(q), _ptr(energy), _ptr(phi), _ptr(dphi), _ptr(hphi), _ptr(gq), _ptr(gQ), _ptr(gmu),
                          _ptr(gth), sel_n, sel_arg, _ptr(gm), _ptr(gmq))
    if rc != 0:
        raise ValueError(f"oracle_ewald rejected its arguments (status {rc})")
    return OracleResult(energy=dict(zip(ENERGY_NAMES, energy.tolist())), phi=phi, dphi=dphi, hphi=hphi,
                        g_qm_pos=gq, g_Q=gQ, g_mu=gmu, g_theta=gth, g_mm_pos=gm, g_mm_q=gmq,
                        mm_sel=None if mm_sel is None else np.asarray(mm_sel))


class _RegionParams(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("r_region", ctypes.c_double),
        ("r_gauss", ctypes.c_double),
    ]


REGION_ENERGY_NAMES = ("qq_bare", "mm_bare", "gauss")


@dataclass
class OracleRegionResult:
    energy: dict           # qq_bare, mm_bare, gauss and their sum under "total"
    phi: np.ndarray        # (nq,)   correction to the MM potential at the QM sites
    dphi: np.ndarray       # (nq,3)  its gradient
    hphi: np.ndarray       # (nq,6)  one half of its Hessian
    g_qm_pos: np.ndarray   # (nq,3)  gradient of the correction energy
    g_Q: np.ndarray
    g_mu: np.ndarray
    g_theta: np.ndarray    # (nq,6)  w.r.t. stored numbers
    g_mm_pos: np.ndarray   # (nm,3)
    g_mm_q: np.ndarray     # (nm,)
    n_region_images: int   # MM lattice translates inside the region-I sphere
    n_gauss_pairs: int     # (QM site, region-II MM translate) pairs of the Gaussian correction

    @property
    def E(self) -> float:
        return self.energy["total"]


def oracle_region(box, r_region, r_gauss, qm_pos, Q, mu, theta, mm_pos, q, kappa=None,
                  lib_path: str | None = None) -> OracleRegionResult:
    """Region-I subtraction and Gaussian-charge correction terms.

    Adding them to :func:`oracle_ewald`'s outputs gives the region-II energy,
    site field and gradients (paper: periodic QM/MM multipole energy and the
    Gaussian-charge correction).  kappa: (nm,) Gaussian exponents, <= 0 or
    None for point charges.
    """
    lib = load(lib_path) if lib_path else load()
    qm_pos = _c(qm_pos).reshape(-1, 3)
    nq = qm_pos.shape[0]
    Q = _c(Q, (nq,))
    mu = _c(mu, (nq, 3))
    theta = _c(theta, (nq, 6))
    mm_pos = _c(mm_pos).reshape(-1, 3)
    nm = mm_pos.shape[0]
    q = _c(q, (nm,))
    kap = None if kappa is None else _c(kappa, (nm,))
    p = _RegionParams()
    p.box[:] = [float(b) for b in box]
    p.r_region = float(r_region)
    p.r_gauss = float(r_gauss)
    energy = np.zeros(3)
    phi = np.zeros(nq)
    dphi = np.zeros((nq, 3))
    hphi = np.zeros((nq, 6))
    gq = np.zeros((nq, 3))
    gQ = np.zeros(nq)
    gmu = np.zeros((nq, 3))
    gth = np.zeros((nq, 6))
    gm = np.zeros((nm, 3))
    gmq = np.zeros(nm)
    counts = np.zeros(2, dtype=np.int64)
    rc = lib.oracle_region(ctypes.byref(p), nq, _ptr(qm_pos), _ptr(Q), _ptr(mu), _ptr(theta), nm, _ptr(mm_pos),
                           _ptr(q), None if kap is None else _ptr(kap), _ptr(energy), _ptr(phi), _ptr(dphi),
                           _ptr(hphi), _ptr(gq), _ptr(gQ), _ptr(gmu), _ptr(gth), _ptr(gm), _ptr(gmq),
                           counts.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    if rc != 0:
        raise ValueError(f"oracle_region rejected its arguments (status {rc})")
    en = dict(zip(REGION_ENERGY_NAMES, energy.tolist()))
    en["total"] = float(sum(energy))
    return OracleRegionResult(energy=en, phi=phi, dphi=dphi, hphi=hphi, g_qm_pos=gq, g_Q=gQ, g_mu=gmu, g_theta=gth,
                              g_mm_pos=gm, g_mm_q=gmq, n_region_images=int(counts[0]), n_gauss_pairs=int(counts[1]))


OCTUPOLE_COMPONENTS = ("xxx", "xxy", "xxz", "xyy", "xyz", "xzz", "yyy", "yyz", "yzz", "zzz")


def oracle_octupole_error(box, qm_pos, omega, mm_pos, q, r_cut, r_outer, lib_path: str | None = None) -> np.ndarray:
    """Charge-octupole error estimate Err(R_cut) for each candidate R_cut
    (paper: Error Control).  omega (nq,10): raw third moments in the order of
    OCTUPOLE_COMPONENTS; region II is R_cut <= |R - C| < r_outer."""
    lib = load(lib_path) if lib_path else load()
    qm_pos = _c(qm_pos).reshape(-1, 3)
    nq = qm_pos.shape[0]
    om = _c(omega, (nq, 10))
    mm_pos = _c(mm_pos).reshape(-1, 3)
    nm = mm_pos.shape[0]
    q = _c(q, (nm,))
    rc = _c(np.atleast_1d(r_cut))
    b = _c(box, (3,))
    err = np.zeros(rc.size)
    st = lib.oracle_octupole_error(_ptr(b), nq, _ptr(qm_pos), _ptr(om), nm, _ptr(mm_pos), _ptr(q), rc.size, _ptr(rc),
                                   float(r_outer), _ptr(err))
    if st != 0:
        raise ValueError(f"oracle_octupole_error rejected its arguments (status {st})")
    return err


def oracle_rcut_pick(r_cut, err, eps, lib_path: str | None = None) -> float:
    """First candidate whose estimate and the next one's are below eps; -1 if none."""
    lib = load(lib_path) if lib_path else load()
    rc = _c(np.atleast_1d(r_cut))
    e = _c(np.atleast_1d(err))
    return float(lib.oracle_rcut_pick(rc.size, _ptr(rc), _ptr(e), float(eps)))
