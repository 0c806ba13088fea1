"""Pins of the oracle's region-I subtraction and Gaussian-charge correction
against facts that do not come from the oracle itself: hand-summed images,
exact Coulomb and erfc sums over point-charge clusters (the multipole
expansion must then be right to third order), the tin-foil surface term of a
neutral cluster, lattice-translation invariance, finite differences and the
two limits of the Gaussian exponent.

Each check returns the worst deviation it saw; the tests compare it with a
tolerance, and the mutation tests run the same checks on broken copies of
the oracle, so every check takes the library path.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.oracle import oracle_ewald, oracle_octupole_error, oracle_rcut_pick, oracle_region


def _z(n, m):
    return np.zeros((n, m))


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    den = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


# ---------------------------------------------------------------- hand-summed images
def region_hand(lib=None):
    """One QM site at the centre of a 10 A cube (Q = 0.7, mu along x) and one MM
    charge q = -0.4 three Angstrom away along x.  Its translates lie at 3, 7,
    sqrt(109) ~ 10.44, 13 ... from the site.  With r_region = 8 region I holds
    the two at 3 and 7 (the second one is the x - L translate); with r_region
    = 5 only the first.  Written out by hand:
        E = -q [Q (1/3 + 1/7) + mu_x (1/9 - 1/49)],  phi = -q (1/3 + 1/7),
        d phi/dx = -q (1/9 - 1/49)."""
    L, Q, q, mx = 10.0, 0.7, -0.4, 0.2
    qm = np.array([[5.0, 5.0, 5.0]])
    mm = np.array([[8.0, 5.0, 5.0]])
    mu = np.array([[mx, 0.0, 0.0]])
    errs = []
    for rr, inv, inv2, n in ((8.0, 1 / 3 + 1 / 7, 1 / 9 - 1 / 49, 2), (5.0, 1 / 3, 1 / 9, 1)):
        r = oracle_region([L] * 3, rr, 0.0, qm, [Q], mu, _z(1, 6), mm, [q], lib_path=lib)
        errs.append(abs(r.energy["mm_bare"] - (-q * (Q * inv + mx * inv2))) / abs(q * Q * inv))
        errs.append(abs(r.phi[0] - (-q * inv)) / abs(q * inv))
        errs.append(_rel(r.dphi[0], [-q * inv2, 0.0, 0.0]))
        errs.append(0.0 if r.n_region_images == n else 1.0)
        # the MM atom's gradient is minus the site's for a single pair set
        errs.append(_rel(r.g_mm_pos[0], -r.g_qm_pos[0]))
    return max(errs)


# ---------------------------------------------------------------- point-charge clusters
def _cluster_system(seed=21):
    """QM sites near the centre of a 60 A box, MM charges within 9 A of it:
    no other translate of an MM atom comes within 30 A, so region I (r_region
    = 12) is the MM atoms themselves and a Gaussian cutoff of 15 A sees only
    them."""
    rng = np.random.default_rng(seed)
    L = 60.0
    c = np.full(3, L / 2)
    qm = c + rng.uniform(-1.5, 1.5, (3, 3))
    dirs = rng.normal(size=(40, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    mm = c + dirs * rng.uniform(3.5, 9.0, (40, 1))
    q = rng.uniform(-0.9, 0.9, 40)
    kappa = rng.uniform(0.25, 0.6, 40)
    # each QM site is a cluster of four charges at R_j + h u_k
    ck = rng.uniform(-0.8, 0.8, (3, 4))
    uk = rng.normal(size=(3, 4, 3))
    return L, qm, mm, q, kappa, ck, uk


def _cluster_moments(ck, uk, h):
    Q = ck.sum(1)
    mu = np.einsum("jk,jka->ja", ck, h * uk)
    full = np.einsum("jk,jka,jkb->jab", ck, h * uk, h * uk)
    th = full[:, [0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
    return Q, mu, th


def _cluster_exact(qm, mm, q, kappa, ck, uk, h, gaussian):
    e = 0.0
    for j in range(qm.shape[0]):
        for k in range(ck.shape[1]):
            p = qm[j] + h * uk[j, k]
            for i in range(mm.shape[0]):
                d = float(np.linalg.norm(p - mm[i]))
                e -= q[i] * ck[j, k] * (math.erfc(kappa[i] * d) / d if gaussian else 1.0 / d)
    return e


def region_cluster(lib=None):
    """The multipole energy of a point-charge cluster differs from its exact
    Coulomb (or erfc) energy by the missing octupole, O(h^3): halving the
    cluster size must divide the difference by 8.  A wrong order-1 or order-2
    tensor leaves an O(h) or O(h^2) difference (ratio 2 or 4).  Returns the
    worst |log2(ratio) - 3|."""
    L, qm, mm, q, kappa, ck, uk = _cluster_system()
    worst = 0.0
    for gaussian in (False, True):
        d = []
        for h in (0.04, 0.02):
            Q, mu, th = _cluster_moments(ck, uk, h)
            if gaussian:
                r = oracle_region([L] * 3, 0.0, 15.0, qm, Q, mu, th, mm, q, kappa, lib_path=lib)
                got = r.energy["gauss"]
            else:
                r = oracle_region([L] * 3, 12.0, 0.0, qm, Q, mu, th, mm, q, lib_path=lib)
                got = r.energy["mm_bare"]
            d.append(got - _cluster_exact(qm, mm, q, kappa, ck, uk, h, gaussian))
        worst = max(worst, abs(math.log2(abs(d[0] / d[1])) - 3.0))
    return worst


# ---------------------------------------------------------------- tin-foil surface term
def region_qq_sphere(lib=None):
    """A neutral QM cluster alone in a large cube.  The Ewald QM-QM energy
    (tin-foil) minus the bare unit-cell pairs leaves the interaction with the
    periodic images; summed over spheres of cells it vanishes up to
    O(d^4/L^5) by cubic symmetry, and the tin-foil sum differs from the
    spherical one by -2 pi |M|^2 / (3V), M = sum (Q R + mu).  Relative deviation."""
    rng = np.random.default_rng(7)
    L = 300.0
    V = L ** 3
    nq = 4
    qm = L / 2 + rng.uniform(-1.5, 1.5, (nq, 3))
    Q = rng.uniform(-0.8, 0.8, nq)
    Q -= Q.mean()
    mu = rng.normal(0, 0.3, (nq, 3))
    th = rng.normal(0, 0.2, (nq, 6))
    ew = oracle_ewald([L] * 3, 0.04, 120.0, 22, qm, Q, mu, th, np.zeros((0, 3)), [], lib_path=lib)
    rg = oracle_region([L] * 3, 10.0, 0.0, qm, Q, mu, th, np.zeros((0, 3)), [], lib_path=lib)
    M = (Q[:, None] * (qm - L / 2)).sum(0) + mu.sum(0)
    ref = -2.0 * math.pi * float(M @ M) / (3.0 * V)
    return abs(ew.E + rg.energy["qq_bare"] - ref) / abs(ref)


# ---------------------------------------------------------------- invariance, differences, limits
def _random_system(seed=4, nq=5, nm=60, box=(20.0, 22.0, 24.0)):
    rng = np.random.default_rng(seed)
    L = np.array(box)
    qm = L / 2 + rng.uniform(-2.0, 2.0, (nq, 3))
    Q = rng.uniform(-0.9, 0.9, nq)
    mu = rng.normal(0, 0.2, (nq, 3))
    th = rng.normal(0, 0.1, (nq, 6))
    mm = rng.random((nm, 3)) * L
    q = rng.uniform(-0.9, 0.9, nm)
    kappa = rng.uniform(0.5, 1.5, nm)
    kappa[::4] = 0.0  # some point charges
    return L, qm, Q, mu, th, mm, q, kappa


_KEYS = ("phi", "dphi", "hphi", "g_qm_pos", "g_Q", "g_mu", "g_theta", "g_mm_pos", "g_mm_q")


def region_translation(lib=None):
    """Moving MM atoms by whole lattice vectors, or every atom by one common
    vector, changes nothing (region I moves with the QM centre; r_region above
    half the box, so several translates of an atom take part)."""
    L, qm, Q, mu, th, mm, q, kappa = _random_system()
    args = dict(lib_path=lib)
    r0 = oracle_region(L, 14.0, 6.0, qm, Q, mu, th, mm, q, kappa, **args)
    rng = np.random.default_rng(1)
    mm2 = mm + rng.integers(-2, 3, mm.shape) * L
    r1 = oracle_region(L, 14.0, 6.0, qm, Q, mu, th, mm2, q, kappa, **args)
    s = np.array([3.3, -7.1, 12.9])
    r2 = oracle_region(L, 14.0, 6.0, qm + s, Q, mu, th, mm + s, q, kappa, **args)
    worst = 0.0
    for r in (r1, r2):
        worst = max(worst, abs(r.E - r0.E) / abs(r0.E))
        for k in _KEYS:
            worst = max(worst, _rel(getattr(r, k), getattr(r0, k)))
        if r.n_region_images != r0.n_region_images or r.n_gauss_pairs != r0.n_gauss_pairs:
            worst = 1.0
    return worst


def region_fd_positions(lib=None, h=1e-4):
    """Central 4-point differences of the correction energy in every QM
    coordinate and a few MM coordinates (no translate crosses the sphere or
    the Gaussian cutoff within the step: the counts are checked)."""
    L, qm, Q, mu, th, mm, q, kappa = _random_system(seed=8)
    args = (L, 14.0, 6.0)
    r0 = oracle_region(*args, qm, Q, mu, th, mm, q, kappa, lib_path=lib)
    cnt = (r0.n_region_images, r0.n_gauss_pairs)

    def E(qp, mp):
        r = oracle_region(*args, qp, Q, mu, th, mp, q, kappa, lib_path=lib)
        if (r.n_region_images, r.n_gauss_pairs) != cnt:
            raise RuntimeError("membership changed within the step")
        return r.E

    worst = 0.0
    for j in range(qm.shape[0]):
        for a in range(3):
            vals = []
            for s in (-2, -1, 1, 2):
                qp = qm.copy()
                qp[j, a] += s * h
                vals.append(E(qp, mm))
            fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
            worst = max(worst, abs(fd - r0.g_qm_pos[j, a]) / max(np.max(np.abs(r0.g_qm_pos)), 1e-30))
    for i in (0, 5, 17, 33):
        for a in range(3):
            vals = []
            for s in (-2, -1, 1, 2):
                mp = mm.copy()
                mp[i, a] += s * h
                vals.append(E(qm, mp))
            fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
            worst = max(worst, abs(fd - r0.g_mm_pos[i, a]) / max(np.max(np.abs(r0.g_mm_pos)), 1e-30))
    return worst


def region_fd_moments(lib=None, h=1e-3):
    """The correction energy is at most quadratic in the moments and linear in
    q: central differences are exact up to rounding."""
    L, qm, Q, mu, th, mm, q, kappa = _random_system(seed=9)
    args = (L, 14.0, 6.0)
    r0 = oracle_region(*args, qm, Q, mu, th, mm, q, kappa, lib_path=lib)

    def E(Qp=Q, mup=mu, thp=th, qp=q):
        return oracle_region(*args, qm, Qp, mup, thp, mm, qp, kappa, lib_path=lib).E

    worst = 0.0
    scale = max(np.max(np.abs(r0.g_Q)), np.max(np.abs(r0.g_mu)), np.max(np.abs(r0.g_theta)))
    for j in range(qm.shape[0]):
        d = Q.copy(); d[j] += h; e1 = E(Qp=d); d[j] -= 2 * h; e2 = E(Qp=d)  # noqa: E702
        worst = max(worst, abs((e1 - e2) / (2 * h) - r0.g_Q[j]) / scale)
        for a in range(3):
            d = mu.copy(); d[j, a] += h; e1 = E(mup=d); d[j, a] -= 2 * h; e2 = E(mup=d)  # noqa: E702
            worst = max(worst, abs((e1 - e2) / (2 * h) - r0.g_mu[j, a]) / scale)
        for t in range(6):
            d = th.copy(); d[j, t] += h; e1 = E(thp=d); d[j, t] -= 2 * h; e2 = E(thp=d)  # noqa: E702
            worst = max(worst, abs((e1 - e2) / (2 * h) - r0.g_theta[j, t]) / scale)
    qs = max(np.max(np.abs(r0.g_mm_q)), 1e-30)
    for i in (1, 4, 9, 30):
        d = q.copy(); d[i] += h; e1 = E(qp=d); d[i] -= 2 * h; e2 = E(qp=d)  # noqa: E702
        worst = max(worst, abs((e1 - e2) / (2 * h) - r0.g_mm_q[i]) / qs)
    return worst


def region_gauss_limits(lib=None):
    """A very tight Gaussian is a point charge: no correction.  A very wide one
    (kappa -> 0, erfc -> 1) turns the correction into minus the bare
    interaction with every region-II translate within r_gauss; with a single
    QM site at the centre that is the region-I subtraction at r_region = r_gauss
    minus the one at the actual r_region."""
    L, qm, Q, mu, th, mm, q, kappa = _random_system(seed=12, nq=1)
    big = oracle_region(L, 9.0, 0.0, qm, Q, mu, th, mm, q, lib_path=lib)
    small = oracle_region(L, 6.0, 0.0, qm, Q, mu, th, mm, q, lib_path=lib)
    tight = oracle_region(L, 6.0, 9.0, qm, Q, mu, th, mm, q, np.full_like(q, 80.0), lib_path=lib)
    e_tight = abs(tight.energy["gauss"]) + float(np.max(np.abs(tight.phi - small.phi)))
    if tight.n_gauss_pairs == 0:
        e_tight = 1.0  # the case must have Gaussian pairs to mean anything
    wide = oracle_region(L, 6.0, 9.0, qm, Q, mu, th, mm, q, np.full_like(q, 1e-10), lib_path=lib)
    ref = big.energy["mm_bare"] - small.energy["mm_bare"]
    e_wide = abs(wide.energy["gauss"] - ref) / abs(ref)
    e_field = _rel(wide.phi - small.phi, big.phi - small.phi)
    return max(e_tight, e_wide, e_field)


# ---------------------------------------------------------------- octupole error estimate
def octupole_hand(lib=None):
    """One site at the centre with a single octupole component w and one
    charge q at offset (a, b, c) from it (r = site - charge = -(a, b, c)).
    The octupole tensor is one sixth of the third derivative of 1/r:
      xxx only, charge on the x axis at distance d:  Err = q w / d^4;
      xyz only (six index orders): Err = 15 q w a b c / r^7.
    Candidates beyond the charge, or an outer radius inside it, give 0."""
    L, q, w = 40.0, 0.7, 0.3
    qm = np.array([[20.0, 20.0, 20.0]])
    errs = []
    d = 3.0
    om = np.zeros((1, 10)); om[0, 0] = w  # noqa: E702
    e = oracle_octupole_error([L] * 3, qm, om, [[23.0, 20.0, 20.0]], [q], [0.0, 2.9, 3.1], 15.0, lib_path=lib)
    errs += [abs(e[0] - q * w / d ** 4) / (q * w / d ** 4), abs(e[1] - e[0]) / abs(e[0]), abs(e[2])]
    a, b, c = 1.2, -0.7, 2.1
    r = math.sqrt(a * a + b * b + c * c)
    om = np.zeros((1, 10)); om[0, 4] = w  # noqa: E702
    e = oracle_octupole_error([L] * 3, qm, om, [[20.0 + a, 20.0 + b, 20.0 + c]], [q], [0.0], 15.0, lib_path=lib)
    ref = 15.0 * q * w * a * b * c / r ** 7
    errs.append(abs(e[0] - ref) / abs(ref))
    e = oracle_octupole_error([L] * 3, qm, om, [[20.0 + a, 20.0 + b, 20.0 + c]], [q], [0.0], 0.5 * r, lib_path=lib)
    errs.append(abs(e[0]))
    return max(errs)


def octupole_cluster(lib=None):
    """Point-charge clusters again: exact Coulomb energy minus the multipole
    energy through quadrupoles is, to leading order, the charge-octupole
    estimate; what remains is O(h^4), so halving h divides it by 16 (a wrong
    octupole tensor leaves O(h^3): ratio 8).  Returns |log2(ratio) - 4|."""
    L, qm, mm, q, kappa, ck, uk = _cluster_system(seed=23)
    d = []
    for h in (0.08, 0.04):
        Q, mu, th = _cluster_moments(ck, uk, h)
        om = np.einsum("jk,jka,jkb,jkc->jabc", ck, h * uk, h * uk, h * uk)
        idx = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2),
               (2, 2, 2)]
        om10 = np.stack([om[:, a, b, c] for a, b, c in idx], axis=1)
        mult2 = -oracle_region([L] * 3, 12.0, 0.0, qm, Q, mu, th, mm, q, lib_path=lib).energy["mm_bare"]
        oct_ = oracle_octupole_error([L] * 3, qm, om10, mm, q, [0.0], 12.0, lib_path=lib)[0]
        exact = -_cluster_exact(qm, mm, q, kappa, ck, uk, h, False)
        d.append(exact - mult2 - oct_)
    return abs(math.log2(abs(d[0] / d[1])) - 4.0)


def rcut_pick(lib=None):
    """The search takes the first candidate whose estimate and the next one's
    are both below eps in magnitude."""
    rc = [13.0, 14.0, 15.0, 16.0, 17.0, 18.0]
    cases = [([5e-4, 1e-4, 3e-4, 1e-4, 5e-5, 1e-5], 2e-4, 16.0),
             ([-5e-4, -1e-4, -1.5e-4, 1e-4, 5e-5, 1e-5], 2e-4, 14.0),
             ([5e-4, 4e-4, 3e-4, 3e-4, 1e-4, 3e-4], 2e-4, -1.0),
             ([1e-6] * 6, 2e-4, 13.0)]
    bad = 0
    for err, eps, want in cases:
        if oracle_rcut_pick(rc, err, eps, lib_path=lib) != want:
            bad += 1
    return float(bad)


def region_boundary_jump(lib=None):
    """An MM charge crossing the region-I sphere.  Inside, the QM code treats
    it exactly (here: QM sites made of point charges, exact Coulomb) and the
    library subtracts its bare multipole term; outside, it is part of the
    multipole Ewald sum only.  The Ewald sums are continuous in the position,
    so the jump of the total energy across the boundary is minus (exact -
    quadrupole-truncated multipole) of that charge: to leading order minus
    its charge-octupole term, i.e. minus the error estimate (paper: Error
    Control, and the smoothness of the energy surface across R_cut).
    Returns |jump + Err| / |Err|."""
    L, qm, mm, q, kappa, ck, uk = _cluster_system(seed=31)
    h = 0.3
    Q, mu, th = _cluster_moments(ck, uk, h)
    om = np.einsum("jk,jka,jkb,jkc->jabc", ck, h * uk, h * uk, h * uk)
    idx = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2),
           (2, 2, 2)]
    om10 = np.stack([om[:, a, b, c] for a, b, c in idx], axis=1)
    rc = 8.0
    C = qm.mean(0)
    e = np.array([0.6, -0.48, 0.64])
    qx = 0.7
    vals = []
    for d in (rc - 1e-7, rc + 1e-7):
        p = C + d * e
        exact_I = 0.0
        if d < rc:
            for j in range(qm.shape[0]):
                for k in range(ck.shape[1]):
                    exact_I += qx * ck[j, k] / float(np.linalg.norm(qm[j] + h * uk[j, k] - p))
        bare = oracle_region([L] * 3, rc, 0.0, qm, Q, mu, th, p[None, :], [qx], lib_path=lib).energy["mm_bare"]
        vals.append(exact_I + bare)
    jump = vals[1] - vals[0]
    err = oracle_octupole_error([L] * 3, qm, om10, (C + (rc + 1e-7) * e)[None, :], [qx], [rc], 20.0,
                                lib_path=lib)[0]
    return abs(jump + err) / abs(err)


REGION_PINS = {
    "region_boundary_jump": (region_boundary_jump, 0.2),
    "octupole_hand": (octupole_hand, 1e-13),
    "octupole_cluster": (octupole_cluster, 0.15),
    "rcut_pick": (rcut_pick, 0.0),
    "region_hand": (region_hand, 1e-13),
    "region_cluster": (region_cluster, 0.15),
    "region_qq_sphere": (region_qq_sphere, 1e-2),
    "region_translation": (region_translation, 1e-11),
    "region_fd_positions": (region_fd_positions, 1e-8),
    "region_fd_moments": (region_fd_moments, 1e-8),
    "region_gauss_limits": (region_gauss_limits, 1e-8),
}
