"""Suggested Ewald parameters (alpha, kmax) for a target accuracy: with them
the truncated sums of the oracle agree with a converged evaluation (two
different alphas agreeing to 1e-15) to within tol, relative, for the energy
and every gradient, at a cutoff of half the box and at one near the box
length (the paper's regime, several lattice images in real space)."""
import numpy as np
import pytest

from oracle.oracle import oracle_ewald
from paper_2408_03273_amd import workloads as wl
from paper_2408_03273_amd.ewald import suggest_params
from paper_2408_03273_amd._lib import EwaldError

KEYS = ("g_qm_pos", "g_Q", "g_mu", "g_theta", "g_mm_pos", "g_mm_q")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


@pytest.fixture(scope="module")
def converged():
    s = wl.random_system(71, 4, 120, box=(12.4, 12.4, 12.4), alpha=0.3, rcut=6.0, kmax=8)
    args = (s.qm_pos, s.Q, s.mu, s.theta, s.mm_pos, s.q)
    ref = oracle_ewald(s.box, 0.6, 11.9, (18, 18, 18), *args)
    ref2 = oracle_ewald(s.box, 0.7, 11.9, (21, 21, 21), *args)
    assert abs(ref.E - ref2.E) <= 1e-13 * abs(ref.E)
    return s, args, ref


@pytest.mark.parametrize("rcut", [6.0, 11.0])
@pytest.mark.parametrize("tol", [1e-5, 1e-8])
def test_suggested_parameters_meet_tolerance(converged, rcut, tol):
    s, args, ref = converged
    alpha, kmax = suggest_params(s.box, rcut, tol)
    r = oracle_ewald(s.box, alpha, rcut, kmax, *args)
    errs = {"E": abs(r.E - ref.E) / abs(ref.E)}
    errs.update({k: _rel(getattr(r, k), getattr(ref, k)) for k in KEYS})
    assert max(errs.values()) <= tol, (alpha, kmax, errs)


def test_tighter_tolerance_gives_larger_parameters():
    a1, k1 = suggest_params((30.0, 31.0, 40.0), 12.0, 1e-5)
    a2, k2 = suggest_params((30.0, 31.0, 40.0), 12.0, 1e-9)
    assert a2 > a1 and all(m2 > m1 for m1, m2 in zip(k1, k2))
    assert k2[2] > k2[0]  # the longer edge needs more vectors


@pytest.mark.parametrize("args", [((10.0, 10.0, 10.0), 5.0, 0.0), ((10.0, 10.0, 10.0), 5.0, 0.5),
                                  ((10.0, -1.0, 10.0), 5.0, 1e-6), ((10.0, 10.0, 10.0), 0.0, 1e-6)])
def test_suggest_rejects_bad_arguments(args):
    with pytest.raises(EwaldError):
        suggest_params(*args)
