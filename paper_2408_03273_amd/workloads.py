"""Seeded synthetic inputs for the multipolar-Ewald coupling.

This module holds random-number recipes only (no Ewald arithmetic).  It is
shared by the tests, the benchmark and the smoke check; both the HIP library
and the CPU oracle receive the arrays it produces.

The paper's own structures (solvated microtubule and chorismate mutase, water
boxes) are not available, so each workload is a seeded stand-in with the
sizes and Ewald parameters of one benchmark configuration:

  c1  cubic 12.4 A, 216 rigid waters (648 MM charges), 3 QM sites, a=0.30, rc=6,  m=8
  c2  cubic 40 A, 6400 waters (19200 MM), 30 QM sites,           a=0.25, rc=10, m=16
  c3  70x70x72 A, 35000 MM charges (>=1 A apart), 40 QM sites,   a=0.22, rc=12, m=24
  c4  64 frames: L~U(35,50) A, N_MM~U{5000..30000}, N_QM~U{10..60}, a=0.25, rc=10, m=20
  c5  16 replicas: cubic 100 A, 100000 MM (>=1 A apart), 80 QM,  a=0.18, rc=12, m=32

Water model (c1, c2): rigid TIP3P-like geometry, O -0.834 e, H +0.417 e,
O-H 0.9572 A, H-O-H 104.52 deg, uniform random centre and uniform random
orientation (random unit quaternion).  QM moments: charges ~U(-0.9,0.9) minus
their mean, dipoles ~N(0,s_mu) per component, quadrupoles drawn as six
symmetric components ~N(0,s_th) then made traceless.  MM atoms closer than
1.0 A to any QM site are rejected (whole water molecules for c1/c2).
Seed of (config c, frame f): numpy PCG64 default_rng(240803273 + 1000 c + f).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

BASE_SEED = 240803273

O_CHARGE = -0.834
H_CHARGE = 0.417
OH_LEN = 0.9572
HOH_DEG = 104.52


@dataclass
class System:
    """One frame: box, Ewald parameters and the QM/MM arrays (float64, AoS)."""
    box: np.ndarray          # (3,)
    alpha: float
    rcut: float
    kmax: tuple              # (mx, my, mz)
    qm_pos: np.ndarray       # (nq,3)
    Q: np.ndarray            # (nq,)
    mu: np.ndarray           # (nq,3)
    theta: np.ndarray        # (nq,6) xx,xy,xz,yy,yz,zz
    mm_pos: np.ndarray       # (nm,3)
    q: np.ndarray            # (nm,)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nq(self) -> int:
        return int(self.qm_pos.shape[0])

    @property
    def nm(self) -> int:
        return int(self.mm_pos.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.box, self.qm_pos, self.Q, self.mu, self.theta, self.mm_pos, self.q):
            h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        h.update(np.array([self.alpha, self.rcut], dtype=np.float64).tobytes())
        h.update(np.array(self.kmax, dtype=np.int64).tobytes())
        return h.hexdigest()

    def params(self) -> dict:
        return dict(box=self.box, alpha=self.alpha, rcut=self.rcut, kmax=self.kmax)

    def arrays(self) -> dict:
        return dict(qm_pos=self.qm_pos, Q=self.Q, mu=self.mu, theta=self.theta, mm_pos=self.mm_pos, q=self.q)


def rng_for(cfg: int, frame: int = 0) -> np.random.Generator:
    return np.random.default_rng(BASE_SEED + 1000 * cfg + frame)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotation matrices from random unit quaternions (Shoemake)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1) * np.sin(2 * np.pi * u2)
    b = np.sqrt(1.0 - u1) * np.cos(2 * np.pi * u2)
    c = np.sqrt(u1) * np.sin(2 * np.pi * u3)
    d = np.sqrt(u1) * np.cos(2 * np.pi * u3)
    w, x, y, z = d, a, b, c
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def water_template() -> np.ndarray:
    """O at the origin, both H in the xy plane, symmetric about +x."""
    h = np.deg2rad(HOH_DEG) / 2.0
    return np.array([[0.0, 0.0, 0.0],
                     [OH_LEN * np.cos(h), OH_LEN * np.sin(h), 0.0],
                     [OH_LEN * np.cos(h), -OH_LEN * np.sin(h), 0.0]])


def periodic_min_dist(points: np.ndarray, centres: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Minimum-image distance from each point to the nearest centre."""
    if len(centres) == 0:
        return np.full(len(points), np.inf)
    d = points[:, None, :] - centres[None, :, :]
    d -= box * np.round(d / box)
    return np.sqrt((d * d).sum(-1)).min(axis=1)


def waters(rng: np.random.Generator, n_waters: int, box: np.ndarray, avoid: np.ndarray, dmin: float = 1.0):
    """n_waters rigid waters, rejecting molecules with any atom within dmin of `avoid`."""
    tmpl = water_template()
    out = []
    got = 0
    while got < n_waters:
        m = (n_waters - got) * 2 + 8
        centre = rng.random((m, 3)) * box
        R = random_rotations(rng, m)
        atoms = centre[:, None, :] + np.einsum("mij,aj->mai", R, tmpl)
        atoms = atoms - box * np.floor(atoms / box)
        ok = periodic_min_dist(atoms.reshape(-1, 3), avoid, box).reshape(m, 3).min(axis=1) >= dmin
        atoms = atoms[ok][: n_waters - got]
        out.append(atoms)
        got += len(atoms)
    atoms = np.concatenate(out, axis=0)
    pos = atoms.reshape(-1, 3)
    q = np.tile(np.array([O_CHARGE, H_CHARGE, H_CHARGE]), n_waters)
    return pos, q


def rsa_points(rng: np.random.Generator, n: int, box: np.ndarray, dmin: float, avoid: np.ndarray | None = None,
               avoid_d: float = 1.0) -> np.ndarray:
    """Random sequential addition of n points in a periodic box with pair distance >= dmin."""
    acc = np.zeros((0, 3))
    bs = np.asarray(box, dtype=np.float64)
    while len(acc) < n:
        need = n - len(acc)
        cand = rng.random((int(need * 1.2) + 16, 3)) * bs
        cand = np.minimum(cand, bs * (1 - 1e-15))
        if avoid is not None and len(avoid):
            cand = cand[periodic_min_dist(cand, avoid, bs) >= avoid_d]
        if dmin > 0 and len(acc):
            tree = cKDTree(acc, boxsize=bs)
            d, _ = tree.query(cand, k=1)
            cand = cand[d >= dmin]
        if dmin > 0 and len(cand) > 1:
            ctree = cKDTree(cand, boxsize=bs)
            pairs = ctree.query_pairs(dmin, output_type="ndarray")
            drop = np.zeros(len(cand), dtype=bool)
            # greedy: keep the lower index of each conflicting pair unless it was dropped already
            for i, j in pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]:
                if not drop[i]:
                    drop[j] = True
            cand = cand[~drop]
        acc = np.concatenate([acc, cand[:need]], axis=0)
    return acc


def qm_cluster(rng: np.random.Generator, n: int, centre: np.ndarray, radius: float, dmin: float = 1.0) -> np.ndarray:
    pts = []
    while len(pts) < n:
        p = centre + (rng.random(3) * 2 - 1) * radius
        if np.linalg.norm(p - centre) > radius:
            continue
        if pts and np.min(np.linalg.norm(np.array(pts) - p, axis=1)) < dmin:
            continue
        pts.append(p)
    return np.array(pts)


def qm_moments(rng: np.random.Generator, n: int, s_mu: float, s_th: float):
    Q = rng.uniform(-0.9, 0.9, n)
    Q -= Q.mean()
    mu = rng.normal(0.0, s_mu, (n, 3))
    th = rng.normal(0.0, s_th, (n, 6))
    tr = (th[:, 0] + th[:, 3] + th[:, 5]) / 3.0
    th[:, 0] -= tr
    th[:, 3] -= tr
    th[:, 5] -= tr
    return Q, mu, th


def neutral_charges(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.uniform(-0.9, 0.9, n)
    q -= q.mean()
    return q


CONFIGS = {
    1: dict(name="c1", box=(12.4, 12.4, 12.4), alpha=0.30, rcut=6.0, kmax=8),
    2: dict(name="c2", box=(40.0, 40.0, 40.0), alpha=0.25, rcut=10.0, kmax=16),
    3: dict(name="c3", box=(70.0, 70.0, 72.0), alpha=0.22, rcut=12.0, kmax=24),
    4: dict(name="c4", box=None, alpha=0.25, rcut=10.0, kmax=20, frames=64),
    5: dict(name="c5", box=(100.0, 100.0, 100.0), alpha=0.18, rcut=12.0, kmax=32, frames=16),
}


def make_config(cfg: int, frame: int = 0, n_mm_override: int | None = None) -> System:
    """Build frame `frame` of configuration `cfg` (1..5)."""
    c = CONFIGS[cfg]
    rng = rng_for(cfg, frame)
    km = (c["kmax"],) * 3
    if cfg == 1:
        box = np.array(c["box"])
        R = random_rotations(rng, 1)[0]
        qm_pos = box / 2 + water_template() @ R.T
        Q, mu, th = qm_moments(rng, 3, 0.1, 0.05)
        mm_pos, q = waters(rng, 216, box, qm_pos)
    elif cfg == 2:
        box = np.array(c["box"])
        qm_pos = qm_cluster(rng, 30, box / 2, 5.0)
        Q, mu, th = qm_moments(rng, 30, 0.15, 0.08)
        mm_pos, q = waters(rng, 6400, box, qm_pos)
    elif cfg == 3:
        box = np.array(c["box"])
        qm_pos = qm_cluster(rng, 40, box / 2, 6.0)
        Q, mu, th = qm_moments(rng, 40, 0.15, 0.08)
        n = 35000 if n_mm_override is None else n_mm_override
        mm_pos = rsa_points(rng, n, box, 1.0, avoid=qm_pos)
        q = neutral_charges(rng, n)
    elif cfg == 4:
        L = rng.uniform(35.0, 50.0)
        box = np.array([L, L, L])
        nm = int(rng.integers(5000, 30001)) if n_mm_override is None else n_mm_override
        nq = int(rng.integers(10, 61))
        qm_pos = qm_cluster(rng, nq, box / 2, 6.0)
        Q, mu, th = qm_moments(rng, nq, 0.15, 0.08)
        mm_pos = rsa_points(rng, nm, box, 0.0, avoid=qm_pos)
        q = neutral_charges(rng, nm)
    elif cfg == 5:
        box = np.array(c["box"])
        qm_pos = qm_cluster(rng, 80, box / 2, 6.0)
        Q, mu, th = qm_moments(rng, 80, 0.15, 0.08)
        n = 100000 if n_mm_override is None else n_mm_override
        mm_pos = rsa_points(rng, n, box, 1.0, avoid=qm_pos)
        q = neutral_charges(rng, n)
    else:
        raise ValueError(cfg)
    s = System(box=np.asarray(box, dtype=np.float64), alpha=c["alpha"], rcut=c["rcut"], kmax=km,
               qm_pos=np.ascontiguousarray(qm_pos), Q=Q, mu=mu, theta=th,
               mm_pos=np.ascontiguousarray(mm_pos), q=np.ascontiguousarray(q),
               name=f"{c['name']}/f{frame}")
    s.meta["density"] = s.nm / float(np.prod(s.box))
    return s


# covalent radii (Angstrom) of H, C, N, O; a Gaussian MM charge takes the
# exponent 1 / r_cov of its element
COVALENT_RADII = (0.31, 0.76, 0.71, 0.66)


def gaussian_exponents(seed: int, nm: int, point_fraction: float = 0.0) -> np.ndarray:
    """Seeded Gaussian exponents kappa_i = 1/r_cov for nm MM charges, element
    drawn uniformly from H, C, N, O; a fraction of them stays point charges
    (kappa = 0)."""
    rng = np.random.default_rng(seed)
    k = 1.0 / np.asarray(COVALENT_RADII)[rng.integers(0, len(COVALENT_RADII), nm)]
    k[rng.random(nm) < point_fraction] = 0.0
    return k


def random_system(seed: int, nq: int, nm: int, box=(20.0, 20.0, 20.0), alpha: float = 0.35, rcut: float = 8.0,
                  kmax=10, neutral: bool = True, traceless: bool = False, s_mu: float = 0.2, s_th: float = 0.1,
                  min_qm_mm: float = 1.0) -> System:
    """Small random system for parity and property tests."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    qm_pos = qm_cluster(rng, nq, box / 2, min(box.min() / 3, 4.0 + nq ** (1 / 3)), dmin=1.0) if nq else np.zeros((0, 3))
    Q = rng.uniform(-0.9, 0.9, nq)
    if neutral and nq:
        Q -= Q.mean()
    mu = rng.normal(0.0, s_mu, (nq, 3))
    th = rng.normal(0.0, s_th, (nq, 6))
    if traceless and nq:
        tr = (th[:, 0] + th[:, 3] + th[:, 5]) / 3.0
        th[:, 0] -= tr
        th[:, 3] -= tr
        th[:, 5] -= tr
    mm_pos = rsa_points(rng, nm, box, 0.0, avoid=qm_pos, avoid_d=min_qm_mm) if nm else np.zeros((0, 3))
    q = rng.uniform(-0.9, 0.9, nm)
    if neutral and nm:
        q -= q.mean()
    km = (kmax,) * 3 if np.isscalar(kmax) else tuple(kmax)
    return System(box=box, alpha=alpha, rcut=rcut, kmax=km, qm_pos=qm_pos, Q=Q, mu=mu, theta=th, mm_pos=mm_pos, q=q,
                  name=f"random/{seed}")
