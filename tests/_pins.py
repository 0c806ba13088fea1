"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each check returns the worst relative deviation it saw; the tests compare it
with a tolerance.  The same checks run against deliberately broken copies of
the oracle in the mutation tests, so every check takes the library path.
"""
from __future__ import annotations

import os

import numpy as np

from oracle.oracle import oracle_ewald
from tests import _brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lattice_constant(name: str) -> float:
    with open(os.path.join(GOLDEN, "lattice_constants.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()[:2]
            if k == name:
                return float(v)
    raise KeyError(name)


def _z(n, m):
    return np.zeros((n, m))


def relerr(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    den = np.max(np.abs(b)) if b.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a - b))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / den)


# ---------------------------------------------------------------- closed forms
def nacl_potential(lib=None):
    """Na+ as the QM site (Q=1) in the conventional rock-salt cell (a=2, r0=1);
    dE/dQ_Na is the crystal potential at the cation, -M_NaCl / r0."""
    na = [(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0)]
    cl = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]
    qm = np.array([na[0]], float)
    mm = np.array(na[1:] + cl, float)
    q = np.array([1, 1, 1, -1, -1, -1, -1], float)
    r = oracle_ewald([2.0] * 3, 2.6, 2.6, 12, qm, [1.0], _z(1, 3), _z(1, 6), mm, q, lib_path=lib)
    return abs(r.g_Q[0] + lattice_constant("nacl_madelung")) / lattice_constant("nacl_madelung")


def cscl_energy(lib=None):
    """Cs (QM, Q=+1) at the origin and Cl (MM, q=-1) at the body centre of a unit cube.
    E_QQ alone is the simple-cubic background sum xi/(2L); E_QQ + E_QMMM plus the
    MM image energy xi/(2L) is the CsCl lattice energy -M_CsCl / r0."""
    L = 1.0
    xi = lattice_constant("sc_wigner_xi")
    r = oracle_ewald([L] * 3, 3.0, 1.9, 14, [[0, 0, 0]], [1.0], _z(1, 3), _z(1, 6), [[0.5, 0.5, 0.5]], [-1.0], lib_path=lib)
    r0 = np.sqrt(3) / 2
    e1 = abs(r.E + xi / (2 * L) + lattice_constant("cscl_madelung") / r0) / (lattice_constant("cscl_madelung") / r0)
    eqq = r.energy["qq_sr"] + r.energy["qq_lr"] + r.energy["qq_self"] + r.energy["qq_bg"]
    e2 = abs(eqq - xi / (2 * L)) / abs(xi / (2 * L))
    return max(e1, e2)


def sc_charge_quadrupole(lib=None):
    """One site with charge Q and isotropic theta = c I in a cubic box (no MM):
    E = Q^2 xi/(2L) + 2 pi Q c / V (the images' Laplacian is the background
    density 4 pi / V); a traceless theta adds nothing by cubic symmetry."""
    L, Q, c = 3.0, 0.7, 0.3
    V = L ** 3
    xi = lattice_constant("sc_wigner_xi")
    th = np.array([[c, 0, 0, c, 0, c]], float)
    r = oracle_ewald([L] * 3, 2.0, 1.45, 14, [[0.3, 0.4, 0.5]], [Q], _z(1, 3), th, np.zeros((0, 3)), [], lib_path=lib)
    ref = Q * Q * xi / (2 * L) + 2 * np.pi * Q * c / V
    e1 = abs(r.E - ref) / abs(ref)
    th2 = np.array([[0.2, 0.1, -0.05, -0.3, 0.07, 0.1]], float)
    r2 = oracle_ewald([L] * 3, 2.0, 1.45, 14, [[0.3, 0.4, 0.5]], [Q], _z(1, 3), th2, np.zeros((0, 3)), [], lib_path=lib)
    e2 = abs(r2.E - Q * Q * xi / (2 * L)) / abs(Q * Q * xi / (2 * L))
    return max(e1, e2)


def dipole_lattice(lib=None):
    """One dipole per simple-cubic cell, tin-foil: E = -2 pi |mu|^2 / (3V),
    dE/dmu = -4 pi mu / (3V)."""
    L = 2.5
    V = L ** 3
    m = np.array([[0.3, -0.2, 0.5]])
    r = oracle_ewald([L] * 3, 2.2, 1.2, 14, [[0.1, 0.2, 0.3]], [0.0], m, _z(1, 6), np.zeros((0, 3)), [], lib_path=lib)
    ref = -2 * np.pi * (m @ m.T)[0, 0] / (3 * V)
    e1 = abs(r.E - ref) / abs(ref)
    e2 = relerr(r.g_mu[0], -4 * np.pi * m[0] / (3 * V))
    return max(e1, e2)


# ---------------------------------------------------------------- brute force
def brute_system(seed, zero_dipole=False):
    rng = np.random.default_rng(seed)
    L = 6.0
    qm = rng.random((2, 3)) * L
    Q = np.array([0.7, -0.7])
    mu = rng.normal(0, 0.3, (2, 3))
    th = rng.normal(0, 0.2, (2, 6))
    mm = rng.random((3, 3)) * L
    q = np.array([0.5, 0.3, -0.8])
    if zero_dipole:
        mu[-1] = -(Q[:, None] * qm).sum(0) - mu[:-1].sum(0)
    return L, qm, Q, mu, th, mm, q


def brute_force(lib=None, seed=5, Ms=(6, 8, 12, 16, 24, 32)):
    L, qm, Q, mu, th, mm, q = brute_system(seed)
    # every pair is closer than rc = 5.9 < L: the oracle takes all images within rc
    r = oracle_ewald([L] * 3, 1.25, 5.9, 22, qm, Q, mu, th, mm, q, lib_path=lib)
    E, phi, dphi, hphi = _brute.tinfoil_limit(L, qm, Q, mu, th, mm, q, Ms=Ms)
    h6 = hphi[:, [0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
    return max(abs(r.E - E) / abs(E), relerr(r.phi, phi), relerr(r.dphi, dphi), relerr(r.hphi, h6))


# ---------------------------------------------------------------- alpha independence
def alpha_system(seed=11):
    rng = np.random.default_rng(seed)
    L = 20.0
    nq, nm = 4, 30
    qm = L / 2 + rng.normal(0, 2.0, (nq, 3))
    Q = rng.uniform(-0.9, 0.9, nq)          # charged QM region
    mu = rng.normal(0, 0.3, (nq, 3))
    th = rng.normal(0, 0.2, (nq, 6))         # not traceless
    mm = rng.random((nm, 3)) * L
    q = rng.uniform(-0.9, 0.9, nm)           # charged MM region
    return L, qm, Q, mu, th, mm, q


def alpha_independence(lib=None, alphas=(0.6, 0.7, 0.8), rc=9.9, m=32):
    L, qm, Q, mu, th, mm, q = alpha_system()
    rs = [oracle_ewald([L] * 3, a, rc, m, qm, Q, mu, th, mm, q, lib_path=lib) for a in alphas]
    worst = 0.0
    for r in rs[1:]:
        for f in ("phi", "dphi", "hphi", "g_qm_pos", "g_Q", "g_mu", "g_theta", "g_mm_pos", "g_mm_q"):
            worst = max(worst, relerr(getattr(r, f), getattr(rs[0], f)))
        worst = max(worst, abs(r.E - rs[0].E) / abs(rs[0].E))
    return worst


# ---------------------------------------------------------------- finite differences
def fd_system(seed=3):
    rng = np.random.default_rng(seed)
    L = 16.0
    nq, nm = 3, 20
    qm = L / 2 + rng.normal(0, 1.5, (nq, 3))
    Q = rng.uniform(-0.9, 0.9, nq)
    mu = rng.normal(0, 0.3, (nq, 3))
    th = rng.normal(0, 0.2, (nq, 6))
    mm = rng.random((nm, 3)) * L
    q = rng.uniform(-0.9, 0.9, nm)
    return L, qm, Q, mu, th, mm, q


def _min_image_dists(L, a, b):
    d = a[:, None, :] - b[None, :, :]
    d -= L * np.round(d / L)
    return np.sqrt((d * d).sum(-1))


def fd_positions(lib=None, h=1e-4, alpha=0.4, rc=7.0, m=10):
    """Central 4-point differences of E in every QM and MM coordinate."""
    L, qm, Q, mu, th, mm, q = fd_system()
    args = ([L] * 3, alpha, rc, m)
    r = oracle_ewald(*args, qm, Q, mu, th, mm, q, lib_path=lib)
    dqm = _min_image_dists(L, qm, mm)
    dqq = _min_image_dists(L, qm, qm)
    if np.any(np.abs(dqm - rc) < 10 * h) or np.any(np.abs(dqq[dqq > 0] - rc) < 10 * h):
        raise RuntimeError("FD system has a pair at the cutoff; pick another seed")

    def E_at(qm_, mm_):
        return oracle_ewald(*args, qm_, Q, mu, th, mm_, q, lib_path=lib).E

    worst = 0.0
    for arr, g in ((qm, r.g_qm_pos), (mm, r.g_mm_pos)):
        fd = np.zeros_like(arr)
        for i in range(arr.shape[0]):
            for c in range(3):
                vals = []
                for s in (-2, -1, 1, 2):
                    a2 = arr.copy()
                    a2[i, c] += s * h
                    vals.append(E_at(a2, mm) if arr is qm else E_at(qm, a2))
                fd[i, c] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        worst = max(worst, relerr(g, fd))
    return worst


def fd_moments(lib=None, h=1e-3):
    """E is at most quadratic in the moments and linear in q: central differences are exact."""
    L, qm, Q, mu, th, mm, q = fd_system()
    args = ([L] * 3, 0.4, 7.0, 10)
    r = oracle_ewald(*args, qm, Q, mu, th, mm, q, lib_path=lib)

    def E_at(Q_=Q, mu_=mu, th_=th, q_=q):
        return oracle_ewald(*args, qm, Q_, mu_, th_, mm, q_, lib_path=lib).E

    worst = 0.0
    for name, arr, g in (("Q", Q, r.g_Q), ("mu", mu, r.g_mu), ("th", th, r.g_theta), ("q", q, r.g_mm_q)):
        fd = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            vp, vm = arr.copy(), arr.copy()
            vp[idx] += h
            vm[idx] -= h
            kw = {"Q": "Q_", "mu": "mu_", "th": "th_", "q": "q_"}[name]
            fd[idx] = (E_at(**{kw: vp}) - E_at(**{kw: vm})) / (2 * h)
        worst = max(worst, relerr(g, fd))
    return worst


# ---------------------------------------------------------------- invariants
def invariants(lib=None):
    """Translation invariance, zero net force, and E_QMMM equal to the moments
    contracted with the returned potential, field gradient and half Hessian."""
    L, qm, Q, mu, th, mm, q = fd_system()
    args = ([L] * 3, 0.4, 7.0, 10)
    r = oracle_ewald(*args, qm, Q, mu, th, mm, q, lib_path=lib)
    shift = np.array([3.3, -1.7, 12.9])
    r2 = oracle_ewald(*args, qm + shift, Q, mu, th, mm + shift, q, lib_path=lib)
    e1 = abs(r2.E - r.E) / abs(r.E)
    e2 = max(relerr(r2.g_qm_pos, r.g_qm_pos), relerr(r2.g_mm_pos, r.g_mm_pos))
    net = r.g_qm_pos.sum(0) + r.g_mm_pos.sum(0)
    e3 = float(np.max(np.abs(net)) / np.max(np.abs(r.g_mm_pos)))
    TH = _brute.full_theta(th)
    H = _brute.full_theta(r.hphi)
    eqmmm = float((Q * r.phi).sum() + (mu * r.dphi).sum() + (TH * H).sum())
    ref = r.energy["qmmm_sr"] + r.energy["qmmm_lr"] + r.energy["qmmm_bg"]
    e4 = abs(eqmmm - ref) / abs(ref)
    return max(e1, e2, e3, e4)


def background_switch(lib=None):
    """Charged QM and MM subsystems with and without the uniform neutralising
    background: the energy differs by -(pi/(2 a^2 V)) Qtot^2 - (pi/(a^2 V))
    Qtot qtot, every QM potential by -(pi/(a^2 V)) qtot, dE/dQ_j by
    -(pi/(a^2 V)) (Qtot + qtot), dE/dq_i by -(pi/(a^2 V)) Qtot, and no force
    changes (a uniform background exerts none)."""
    L, qm, Q, mu, th, mm, q = fd_system()
    Q = Q + 0.37   # net charges of both subsystems
    q = q - 0.21
    a = 0.4
    args = ([L] * 3, a, 7.0, 10)
    on = oracle_ewald(*args, qm, Q, mu, th, mm, q, lib_path=lib)
    off = oracle_ewald(*args, qm, Q, mu, th, mm, q, lib_path=lib, background=False)
    c = -np.pi / (a * a * L ** 3)
    Qt, qt = float(Q.sum()), float(q.sum())
    e1 = abs((on.E - off.E) - (0.5 * c * Qt * Qt + c * Qt * qt)) / abs(on.E)
    e2 = relerr(on.phi - off.phi, np.full(len(Q), c * qt))
    e3 = relerr(on.g_Q - off.g_Q, np.full(len(Q), c * (Qt + qt)))
    e4 = relerr(on.g_mm_q - off.g_mm_q, np.full(len(q), c * Qt))
    e5 = max(float(np.max(np.abs(on.g_qm_pos - off.g_qm_pos))), float(np.max(np.abs(on.g_mm_pos - off.g_mm_pos)))) \
        / float(np.max(np.abs(on.g_mm_pos)))
    return max(e1, e2, e3, e4, e5)


ALL_PINS = {
    "nacl_potential": (nacl_potential, 1e-9),
    "cscl_energy": (cscl_energy, 1e-9),
    "sc_charge_quadrupole": (sc_charge_quadrupole, 1e-9),
    "dipole_lattice": (dipole_lattice, 1e-9),
    "brute_force": (brute_force, 1e-7),
    "alpha_independence": (alpha_independence, 1e-10),
    "fd_positions": (fd_positions, 1e-8),
    "fd_moments": (fd_moments, 1e-8),
    "invariants": (invariants, 1e-11),
    "background_switch": (background_switch, 1e-11),
}
