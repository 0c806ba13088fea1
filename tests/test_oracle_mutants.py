"""Plant one plausible mistake at a time in a private copy of the oracle
source (dropped factor, flipped sign, swapped operand) and check that at
least one pin catches it.  The committed oracle is never modified."""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as orc
from tests import _pins, _region_pins

# (description, exact text in the oracle source, replacement[, which occurrence])
MUTANTS = [
    ("drop 2 in dipole force (QM side)", "g += mu[3 * j + a] * 2.0 * p2[a][c];", "g += mu[3 * j + a] * p2[a][c];", 0),
    ("drop 2 in dipole force (MM side)", "g += mu[3 * j + a] * 2.0 * p2[a][c];", "g += mu[3 * j + a] * p2[a][c];", 1),
    ("drop 3 in quadrupole force (QM side)", "g += th[a][b] * 3.0 * p3[a][b][c];", "g += th[a][b] * p3[a][b][c];", 0),
    ("drop 3 in quadrupole force (MM side)", "g += th[a][b] * 3.0 * p3[a][b][c];", "g += th[a][b] * p3[a][b][c];", 1),
    ("dipole structure factor sign", "br += -kmu * ei;", "br += kmu * ei;"),
    ("quadrupole structure factor 1/2", "cr_ += -0.5 * kthk * er;", "cr_ += -1.0 * kthk * er;"),
    ("dipole self-energy sign", "- 2.0 * al * al * al / (3.0 * sp) * mm2", "+ 2.0 * al * al * al / (3.0 * sp) * mm2"),
    ("charge-quadrupole self term dropped", "+ 2.0 * al * al * al / (3.0 * sp) * Q[j] * tr;", ";"),
    ("dipole-dipole pair sign", "Pv -= 2.0 * ma[c] * p2[c][d] * mb[d];", "Pv += 2.0 * ma[c] * p2[c][d] * mb[d];", 0),
    ("charge-dipole operands swapped", "Pv += (Qb * ma[c] - Qa * mb[c]) * p1[c];", "Pv += (Qa * ma[c] - Qb * mb[c]) * p1[c];", 0),
    ("charge-quadrupole pair half", "Pv += (Qb * tha[c][d] + Qa * thb[c][d]) * p2[c][d];", "Pv += 0.5 * (Qb * tha[c][d] + Qa * thb[c][d]) * p2[c][d];", 0),
    ("background factor", "P->background ? -PI / (al * al * V) : 0.0;", "P->background ? -PI / (2.0 * al * al * V) : 0.0;"),
    ("f5 coefficient", "f[2] = (f[1] + 4.0 / 3.0 * kappa", "f[2] = (f[1] + 2.0 / 3.0 * kappa"),
    ("f7 coefficient", "f[3] = (f[2] + 8.0 / 15.0 * pow(kappa, 5)", "f[3] = (f[2] + 4.0 / 15.0 * pow(kappa, 5)"),
    ("half in order-2 real tensor", "p2[a][b] = 0.5 * (3.0 * r[a] * r[b] * f[2]", "p2[a][b] = (3.0 * r[a] * r[b] * f[2]"),
    ("MM real-space force sign", "lg[c] -= q[i] * g; /* r depends on -R_mm */", "lg[c] += q[i] * g;"),
    ("order-2 reciprocal projection", "lp[4] += -0.5 * w * kk[0] * kk[0] * yr;", "lp[4] += -1.0 * w * kk[0] * kk[0] * yr;"),
    ("half-space weight", "const double pref = 8.0 * PI / V;", "const double pref = 4.0 * PI / V;"),
    ("reciprocal MM force component", "for (int g = 0; g < 3; g++) lg[g] += w * q[i] * kk[g] * vi;", "for (int g = 0; g < 3; g++) lg[g] += w * q[i] * kk[(g + 1) % 3] * vi;"),
    ("QM-QM LR gradient sign", "for (int g = 0; g < 3; g++) lg[g] += w * kk[g] * (-zi);", "for (int g = 0; g < 3; g++) lg[g] += w * kk[g] * (zi);"),
]

# mistakes in the region-I subtraction and the Gaussian-charge correction
REGION_MUTANTS = [
    ("region-I subtraction sign", "region_pair(r, 0.0, -1.0, q[i]", "region_pair(r, 0.0, 1.0, q[i]"),
    ("region MM force sign", "gm4[c] -= s * qi * g;", "gm4[c] += s * qi * g;"),
    ("region dE/dq sign", "gm4[3] += s * en;", "gm4[3] += en;"),
    ("region dipole force factor", "g += mj[a] * 2.0 * p2[a][c];", "g += mj[a] * p2[a][c];"),
    ("region-I minimum image only", "N[a] = (int)ceil((R1 + fabs(Ri[a] - C[a])) / L[a]) + 1;", "N[a] = 0;"),
    ("Gaussian pairs not excluded from region I", "if (norm3(dC) < R1) continue; /* region I: already direct */", ";"),
    ("Gaussian exponent doubled", "region_pair(r, kappa[i], -1.0", "region_pair(r, 2.0 * kappa[i], -1.0"),
    ("region centre at the origin", "C[a] = nq > 0 ? C[a] / nq : 0.0;", "C[a] = 0.0;", 0),
    ("octupole centre at the origin", "C[a] = nq > 0 ? C[a] / nq : 0.0;", "C[a] = 0.0;", 1),
    ("bare QM-QM half", "e_qq += -0.5L * Pv;", "e_qq += -1.0L * Pv;"),
    ("bare QM-QM dipole-dipole sign", "Pv -= 2.0 * ma[c] * p2[c][d] * mb[d];", "Pv += 2.0 * ma[c] * p2[c][d] * mb[d];", 1),
    ("bare QM-QM charge-dipole operands swapped", "Pv += (Qb * ma[c] - Qa * mb[c]) * p1[c];",
     "Pv += (Qa * ma[c] - Qb * mb[c]) * p1[c];", 1),
    ("bare QM-QM charge-quadrupole half", "Pv += (Qb * tha[c][d] + Qa * thb[c][d]) * p2[c][d];",
     "Pv += 0.5 * (Qb * tha[c][d] + Qa * thb[c][d]) * p2[c][d];", 1),
    ("octupole tensor sign", "double T = -(5.0 * r[a] * r[b] * r[c] - r2 * dd) / (2.0 * r7);",
     "double T = (5.0 * r[a] * r[b] * r[c] - r2 * dd) / (2.0 * r7);"),
    ("octupole tensor trace term", "double T = -(5.0 * r[a] * r[b] * r[c] - r2 * dd) / (2.0 * r7);",
     "double T = -(5.0 * r[a] * r[b] * r[c] - 3.0 * r2 * dd) / (2.0 * r7);"),
    ("octupole component order", "{{1, 3, 4}, {3, 6, 7}, {4, 7, 8}},", "{{1, 3, 4}, {3, 6, 8}, {4, 8, 7}},"),
    ("octupole region-II inner bound", "if (!(D >= r_cut[k] && D < r_outer)) continue;",
     "if (!(D < r_outer)) continue;"),
    ("R_cut search takes one passing value", "if (fabs(err[k]) < eps && fabs(err[k + 1]) < eps) return r_cut[k];",
     "if (fabs(err[k]) < eps) return r_cut[k];"),
    ("bare QM-QM theta gradient", "agm[10 * a + 4 + sym6(c, d)] += -0.5L * Qb * p2[c][d];",
     "agm[10 * a + 4 + sym6(c, d)] += -0.25L * Qb * p2[c][d];"),
]

FAST_PINS = ["nacl_potential", "sc_charge_quadrupole", "dipole_lattice", "alpha_independence", "fd_positions",
             "fd_moments", "invariants", "brute_force"]


@pytest.fixture(scope="module")
def src_text():
    with open(orc._SRC) as f:
        return f.read()


def _apply(text, old, new, occurrence):
    pos = -1
    for _ in range(occurrence + 1):
        pos = text.index(old, pos + 1)
    return text[:pos] + new + text[pos + len(old):]


def _region_pins_caught(so):
    for name, (fn, tol) in _region_pins.REGION_PINS.items():
        try:
            err = fn(lib=so)
        except Exception as e:  # a crash or a rejected input also counts as caught
            return f"{name}: {type(e).__name__}"
        if not (err <= tol):
            return f"{name}: {err:.2e}"
    return None


@pytest.mark.parametrize("mut", REGION_MUTANTS, ids=[m[0] for m in REGION_MUTANTS])
def test_region_mutant_is_caught(mut, src_text, tmp_path):
    desc, old, new = mut[:3]
    occurrence = mut[3] if len(mut) > 3 else None
    n = src_text.count(old)
    if occurrence is None:
        assert n == 1, f"mutation anchor not unique/found: {old!r}"
        occurrence = 0
    else:
        assert n > occurrence, f"mutation anchor occurrence {occurrence} missing: {old!r}"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(_apply(src_text, old, new, occurrence))
    so = str(tmp_path / "libmutant.so")
    orc.build(src=str(msrc), out=so)
    caught = _region_pins_caught(so)
    assert caught, f"mutant '{desc}' passed every region pin"


@pytest.mark.parametrize("mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(mut, src_text, tmp_path):
    desc, old, new = mut[:3]
    occurrence = mut[3] if len(mut) > 3 else None
    n = src_text.count(old)
    if occurrence is None:
        assert n == 1, f"mutation anchor not unique/found: {old!r}"
        occurrence = 0
    else:
        assert n > occurrence, f"mutation anchor occurrence {occurrence} missing: {old!r}"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(_apply(src_text, old, new, occurrence))
    so = str(tmp_path / "libmutant.so")
    orc.build(src=str(msrc), out=so)
    caught = []
    for name in FAST_PINS:
        fn, tol = _pins.ALL_PINS[name]
        try:
            if name == "brute_force":
                err = fn(lib=so, Ms=(6, 8, 12, 16))
                tol = 1e-5
            else:
                err = fn(lib=so)
        except Exception as e:  # a crash or a rejected input also counts as caught
            caught.append(f"{name}: {type(e).__name__}")
            break
        if not (err <= tol):
            caught.append(f"{name}: {err:.2e}")
            break
    assert caught, f"mutant '{desc}' passed every pin"
