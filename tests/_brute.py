"""Direct lattice sums of bare point-multipole interactions (test helper).

Written independently of the oracle: bare Coulomb Taylor coefficients
T = 1/R, T_a = -R_a/R^3, T_ab = (3 R_a R_b - delta_ab R^2)/(2 R^5) (SI, point
multipole interaction tensors) summed over a cube of (2M+1)^3 images of a
small cubic cell, then extrapolated in M.  For a cubic cell, summing whole
cells over a growing cube has the same shape term as a sphere, so the
tin-foil lattice sum is the cube limit minus (2 pi / 3V)|M_cell|^2; with the
MM-MM part excluded and each subsystem neutral this is
(2 pi / 3V)(|M_QM|^2 + 2 M_QM . M_MM), with M_QM = sum_j (Q_j R_j + mu_j) and
M_MM = sum_i q_i R_i.  For the MM potential at a QM site the cube limit and
the tin-foil value differ by (2 pi / 3V) sum_i q_i |R_i - R_j|^2 (shape term
plus the mean-potential term of neutral cells), so the field picks up
-(4 pi / 3V) M_MM and the half Hessian nothing.
"""
from __future__ import annotations

import numpy as np

_SYM = np.array([[0, 1, 2], [1, 3, 4], [2, 4, 5]])


def full_theta(th6):
    return np.asarray(th6)[..., _SYM]


def bare_tensors(R):
    r2 = (R * R).sum(-1)
    r = np.sqrt(r2)
    T0 = 1.0 / r
    T1 = -R / r[..., None] ** 3
    T2 = (3.0 * R[..., :, None] * R[..., None, :] - np.eye(3) * r2[..., None, None]) / (2.0 * r[..., None, None] ** 5)
    return T0, T1, T2


def image_vectors(L, M):
    n = np.arange(-M, M + 1)
    return np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3) * L


def cube_sums(L, M, qm, Q, mu, th6, mm, q):
    """E_QQ + E_QMMM over a cube of images, and the MM potential data at QM sites."""
    Ls = image_vectors(L, M)
    TH = full_theta(th6)
    nq = len(Q)
    E = 0.0
    phi = np.zeros(nq)
    dphi = np.zeros((nq, 3))
    hphi = np.zeros((nq, 3, 3))
    for a in range(nq):
        for b in range(nq):
            R = qm[a] - qm[b] + Ls
            if a == b:
                R = R[np.any(Ls != 0, axis=1)]
            T0, T1, T2 = bare_tensors(R)
            P = (Q[a] * Q[b] * T0 + ((Q[b] * mu[a] - Q[a] * mu[b]) * T1).sum(-1)
                 + ((Q[b] * TH[a] + Q[a] * TH[b]) * T2).sum((-1, -2))
                 - 2.0 * np.einsum("i,nij,j->n", mu[a], T2, mu[b]))
            E += 0.5 * P.sum()
        for i in range(len(q)):
            R = qm[a] - mm[i] + Ls
            T0, T1, T2 = bare_tensors(R)
            phi[a] += q[i] * T0.sum()
            dphi[a] += q[i] * T1.sum(0)
            hphi[a] += q[i] * T2.sum(0)
    for a in range(nq):
        E += Q[a] * phi[a] + mu[a] @ dphi[a] + (TH[a] * hphi[a]).sum()
    return E, phi, dphi, hphi


def tinfoil_limit(L, qm, Q, mu, th6, mm, q, Ms=(6, 8, 12, 16, 24, 32), powers=(2, 3, 4, 5)):
    """Extrapolate the cube sums to M -> infinity and apply the tin-foil surface term."""
    qm, mm = np.asarray(qm, float), np.asarray(mm, float)
    Q, q, mu = np.asarray(Q, float), np.asarray(q, float), np.asarray(mu, float)
    V = L ** 3
    MQ = (Q[:, None] * qm).sum(0) + mu.sum(0)
    MM = (q[:, None] * mm).sum(0) if len(q) else np.zeros(3)
    res = [cube_sums(L, M, qm, Q, mu, th6, mm, q) for M in Ms]
    Mv = np.array(Ms, float)
    A = np.vstack([np.ones_like(Mv)] + [Mv ** -p for p in powers]).T

    def extrap(vals):
        vals = np.asarray(vals)
        flat = vals.reshape(len(Ms), -1)
        c = np.linalg.lstsq(A, flat, rcond=None)[0]
        return c[0].reshape(vals.shape[1:])

    E = float(extrap([r[0] for r in res])) - 2 * np.pi / (3 * V) * (MQ @ MQ + 2 * MQ @ MM)
    d2 = ((qm[:, None, :] - mm[None, :, :]) ** 2).sum(-1) if len(q) else np.zeros((len(Q), 0))
    phi = extrap([r[1] for r in res]) + 2 * np.pi / (3 * V) * (d2 @ q)
    dphi = extrap([r[2] for r in res]) - 4 * np.pi / (3 * V) * MM[None, :]
    hphi = extrap([r[3] for r in res])
    return E, phi, dphi, hphi
