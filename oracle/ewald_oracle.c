/*
 * Plain FP64 CPU oracle for the periodic (Ewald) electrostatic coupling of
 * atom-centred QM point multipoles (charge Q, dipole mu, raw second moment
 * theta) with MM point charges q, in an orthorhombic box with tin-foil
 * boundary conditions.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP library is
 * checked against; it is loaded by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark, and by nothing else.  It shares no code,
 * header, table or constant with the GPU path.
 *
 * What is computed (paper: Methods, "Multipole Approximation to
 * Electrostatics", the periodic energy expression, and the Supporting
 * Information section "Multipolar Ewald"):
 *
 *   E = E_QMMM + E_QQ
 *   E_QMMM = sum_j [ Q_j phi_j + mu_j . grad phi_j + theta_j : (1/2) grad grad phi_j ]
 *            phi_j = sum_i q_i psi(R_j - R_i)   (Ewald potential of the MM charges)
 *   E_QQ   = 1/2 sum_{a,b,L}' P(a, b + L)  truncated at total multipole order 2
 *            (charge-charge, charge-dipole, charge-quadrupole, dipole-dipole)
 *
 * with psi = psi_SR + psi_LR + psi_background and the interaction tensors
 * being Taylor coefficients of the Coulomb kernel: order 0 the value, order 1
 * the gradient with respect to the QM position, order 2 one half of the
 * Hessian, order 3 one sixth of the third derivative (SI, definitions of
 * T, T_a, T_ab, T_abc and their screened counterparts with f1, f3, f5, f7).
 * MM-MM interactions are not part of this quantity (Implementation section).
 *
 * Readings of the paper that this oracle freezes (each is listed in the
 * design notes of the repository):
 *  - theta is the raw (not traceless) Cartesian second moment; the 1/2 of the
 *    Taylor series lives in the order-2 tensor, so theta enters S(k) as
 *    -1/2 k.theta.k.
 *  - The order-2 reciprocal tensor is -(2 pi / V) sum_G g(G) e^{...} G_a G_b,
 *    i.e. one half of the second derivative of the order-0 lattice sum.
 *  - Self terms are derived from first principles as minus one half of the
 *    interaction of each multipole with its own screening Gaussian:
 *    -(a/sqrt(pi)) Q^2 - (2 a^3 / (3 sqrt(pi))) |mu|^2 + (2 a^3/(3 sqrt(pi))) Q tr(theta).
 *  - The QM-QM pair form uses both orientations of each pair:
 *    P = Qa Qb psi0 + (Qb mu_a - Qa mu_b).psi1 + (Qb th_a + Qa th_b):psi2
 *        - 2 mu_a.psi2.mu_b.
 *  - A uniform neutralising background is included for charged subsystems:
 *    -(pi/(2 a^2 V)) Qtot^2 (QM-QM) and -(pi/(a^2 V)) Qtot qtot (QM-MM)
 *    (the paper is silent; params.background = 0 leaves both out).
 *  - k-set: every n with |n_x|<=mx, |n_y|<=my, |n_z|<=mz, n != 0, taken as
 *    the half-space nx>0 | (nx=0 & ny>0) | (nx=ny=0 & nz>0) with weight 2.
 *  - Real space: every lattice image with |r| < rcut (strict), all images.
 *
 * oracle_region (end of file) adds the region-I / region-II split: the bare
 * direct sums over region I that the SCF quantities subtract from the Ewald
 * sums, and the Gaussian-smeared MM charge correction.
 *
 * Summation uses long double accumulators.  Phases e^{i k.R} are formed as
 * the product of three per-axis factors, each evaluated directly with
 * cos/sin of n*2*pi*x/L (no recurrences).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846264338327950288

typedef struct {
  double box[3];
  double alpha;
  double rcut;
  int kmax[3];
  int qmqm;       /* include the QM-QM image terms */
  int background; /* include the uniform neutralising background terms */
} oracle_params_t;

enum {
  EN_TOTAL = 0,
  EN_QMMM_SR,
  EN_QMMM_LR,
  EN_QMMM_BG,
  EN_QQ_SR,
  EN_QQ_LR,
  EN_QQ_SELF,
  EN_QQ_BG,
  EN_COUNT
};

/* index of the full symmetric 3x3 component (a,b) in the 6-vector
 * (xx, xy, xz, yy, yz, zz) */
static int sym6(int a, int b) {
  static const int m[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return m[a][b];
}

/* Screened radial functions f1..f7 (SI, "Multipolar Ewald"), kappa = alpha. */
static void radial_f(double r, double kappa, double f[4]) {
  double r2 = r * r;
  double e = exp(-kappa * kappa * r2);
  double sp = sqrt(PI);
  f[0] = erfc(kappa * r) / r;                                              /* f1 */
  f[1] = (f[0] + 2.0 * kappa / sp * e) / r2;                               /* f3 */
  f[2] = (f[1] + 4.0 / 3.0 * kappa * kappa * kappa / sp * e) / r2;         /* f5 */
  f[3] = (f[2] + 8.0 / 15.0 * pow(kappa, 5) / sp * e) / r2;                /* f7 */
}

/* Real-space tensors of erfc(kappa r)/r about the QM centre, r = R_qm - R_other:
 *  p0 = f1
 *  p1[a] = -r_a f3
 *  p2[a][b] = 1/2 (3 r_a r_b f5 - delta_ab f3)
 *  p3[a][b][c] = 1/2 [ (delta_ab r_c + delta_ac r_b + delta_bc r_a) f5 - 5 r_a r_b r_c f7 ]
 * These are the screened T, T_a, T_ab, T_abc written with f3 instead of the
 * explicit Gaussian terms (the two forms are algebraically identical).
 */
static void real_tensors(const double r[3], double kappa, double* p0, double p1[3], double p2[3][3],
                         double p3[3][3][3]) {
  double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  double f[4];
  radial_f(d, kappa, f);
  *p0 = f[0];
  for (int a = 0; a < 3; a++) p1[a] = -r[a] * f[1];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) p2[a][b] = 0.5 * (3.0 * r[a] * r[b] * f[2] - (a == b ? f[1] : 0.0));
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      for (int c = 0; c < 3; c++) {
        double s = 0.0;
        if (a == b) s += r[c];
        if (a == c) s += r[b];
        if (b == c) s += r[a];
        p3[a][b][c] = 0.5 * (s * f[2] - 5.0 * r[a] * r[b] * r[c] * f[3]);
      }
}

/* full symmetric matrix from the 6 stored numbers */
static void unpack_sym(const double* t6, double t[3][3]) {
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) t[a][b] = t6[sym6(a, b)];
}

/* Accumulate d/d(stored theta component) given dE/dtheta_ab for the full
 * symmetric matrix: off-diagonal stored numbers appear twice. */
static void add_theta_grad(double* g6, double full[3][3], double scale) {
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) g6[sym6(a, b)] += scale * full[a][b];
}

static int image_range(double rc, double L) { return (int)ceil(rc / L) + 1; }

int oracle_ewald(const oracle_params_t* P, int nq, const double* qm_pos, const double* Q, const double* mu,
                 const double* theta, int nm, const double* mm_pos, const double* q,
                 double* energy,      /* EN_COUNT */
                 double* phi,         /* nq */
                 double* dphi,        /* nq*3  grad phi */
                 double* hphi,        /* nq*6  1/2 grad grad phi (xx,xy,xz,yy,yz,zz) */
                 double* g_qm_pos,    /* nq*3  dE/dR_qm */
                 double* g_Q,         /* nq */
                 double* g_mu,        /* nq*3 */
                 double* g_theta,     /* nq*6  w.r.t. the stored numbers */
                 int n_sel, const int* mm_sel, /* MM atoms that get gradients; n_sel<0: all */
                 double* g_mm_pos,    /* n_sel*3 (or nm*3) */
                 double* g_mm_q)      /* n_sel (or nm) */
{
  const double Lx = P->box[0], Ly = P->box[1], Lz = P->box[2];
  const double V = Lx * Ly * Lz;
  const double al = P->alpha, rc = P->rcut;
  const int mx = P->kmax[0], my = P->kmax[1], mz = P->kmax[2];
  if (nq < 0 || nm < 0 || al <= 0.0 || rc <= 0.0 || Lx <= 0.0 || Ly <= 0.0 || Lz <= 0.0 || mx < 0 ||
      my < 0 || mz < 0)
    return -1;
  const int nsel = (n_sel < 0) ? nm : n_sel;
  const double L[3] = {Lx, Ly, Lz};
  /* 0. wrap positions into the reference cell (the sums are periodic) */
  double* wq = malloc(sizeof(double) * 3 * (size_t)(nq > 0 ? nq : 1));
  double* wm = malloc(sizeof(double) * 3 * (size_t)(nm > 0 ? nm : 1));
  for (int j = 0; j < nq; j++)
    for (int a = 0; a < 3; a++) wq[3 * j + a] = qm_pos[3 * j + a] - L[a] * floor(qm_pos[3 * j + a] / L[a]);
  for (int i = 0; i < nm; i++)
    for (int a = 0; a < 3; a++) wm[3 * i + a] = mm_pos[3 * i + a] - L[a] * floor(mm_pos[3 * i + a] / L[a]);
  qm_pos = wq;
  mm_pos = wm;
  const double sp = sqrt(PI);

  long double en[EN_COUNT];
  for (int e = 0; e < EN_COUNT; e++) en[e] = 0.0L;

  /* per-QM-site accumulators */
  long double* aphi = calloc((size_t)nq * 10, sizeof(long double)); /* phi, dphi[3], hphi[6] */
  long double* agq = calloc((size_t)nq * 3, sizeof(long double));   /* dE/dR_qm */
  long double* agm = calloc((size_t)nq * 10, sizeof(long double));  /* QM-QM part of dE/dQ,dmu,dtheta(full: xx..zz as 6) */
  long double* agmm = calloc((size_t)(nsel > 0 ? nsel : 1) * 4, sizeof(long double));

  double qtot = 0.0, Qtot = 0.0;
  for (int i = 0; i < nm; i++) qtot += q[i];
  for (int j = 0; j < nq; j++) Qtot += Q[j];

  const int nix = image_range(rc, Lx), niy = image_range(rc, Ly), niz = image_range(rc, Lz);

  /* ---------- 1. QM-MM real space (SI: screened tensors with kappa = alpha) ---------- */
  /* QM-side sums: parallel over QM sites */
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j < nq; j++) {
    double th[3][3];
    unpack_sym(theta + 6 * j, th);
    long double lphi[10] = {0}, lg[3] = {0}, le = 0.0L;
    for (int i = 0; i < nm; i++) {
      for (int ix = -nix; ix <= nix; ix++)
        for (int iy = -niy; iy <= niy; iy++)
          for (int iz = -niz; iz <= niz; iz++) {
            double r[3] = {qm_pos[3 * j + 0] - mm_pos[3 * i + 0] + ix * Lx,
                           qm_pos[3 * j + 1] - mm_pos[3 * i + 1] + iy * Ly,
                           qm_pos[3 * j + 2] - mm_pos[3 * i + 2] + iz * Lz};
            double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (!(d2 < rc * rc)) continue;
            double p0, p1[3], p2[3][3], p3[3][3][3];
            real_tensors(r, al, &p0, p1, p2, p3);
            double qi = q[i];
            lphi[0] += qi * p0;
            for (int a = 0; a < 3; a++) lphi[1 + a] += qi * p1[a];
            lphi[4] += qi * p2[0][0];
            lphi[5] += qi * p2[0][1];
            lphi[6] += qi * p2[0][2];
            lphi[7] += qi * p2[1][1];
            lphi[8] += qi * p2[1][2];
            lphi[9] += qi * p2[2][2];
            double e = Q[j] * p0;
            for (int a = 0; a < 3; a++) e += mu[3 * j + a] * p1[a];
            for (int a = 0; a < 3; a++)
              for (int b = 0; b < 3; b++) e += th[a][b] * p2[a][b];
            le += qi * e;
            /* dE/dR_qm: d p0/dr_c = p1_c, d p1_a/dr_c = 2 p2_ac, d p2_ab/dr_c = 3 p3_abc */
            for (int c = 0; c < 3; c++) {
              double g = Q[j] * p1[c];
              for (int a = 0; a < 3; a++) g += mu[3 * j + a] * 2.0 * p2[a][c];
              for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) g += th[a][b] * 3.0 * p3[a][b][c];
              lg[c] += qi * g;
            }
          }
    }
    for (int t = 0; t < 10; t++) aphi[10 * j + t] += lphi[t];
    for (int c = 0; c < 3; c++) agq[3 * j + c] += lg[c];
#pragma omp critical
    en[EN_QMMM_SR] += le;
  }
  /* MM-side sums: parallel over the selected MM atoms */
#pragma omp parallel for schedule(dynamic, 64)
  for (int s = 0; s < nsel; s++) {
    int i = (n_sel < 0) ? s : mm_sel[s];
    long double lg[3] = {0}, lq = 0.0L;
    for (int j = 0; j < nq; j++) {
      double th[3][3];
      unpack_sym(theta + 6 * j, th);
      for (int ix = -nix; ix <= nix; ix++)
        for (int iy = -niy; iy <= niy; iy++)
          for (int iz = -niz; iz <= niz; iz++) {
            double r[3] = {qm_pos[3 * j + 0] - mm_pos[3 * i + 0] + ix * Lx,
                           qm_pos[3 * j + 1] - mm_pos[3 * i + 1] + iy * Ly,
                           qm_pos[3 * j + 2] - mm_pos[3 * i + 2] + iz * Lz};
            double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (!(d2 < rc * rc)) continue;
            double p0, p1[3], p2[3][3], p3[3][3][3];
            real_tensors(r, al, &p0, p1, p2, p3);
            double e = Q[j] * p0;
            for (int a = 0; a < 3; a++) e += mu[3 * j + a] * p1[a];
            for (int a = 0; a < 3; a++)
              for (int b = 0; b < 3; b++) e += th[a][b] * p2[a][b];
            lq += e;
            for (int c = 0; c < 3; c++) {
              double g = Q[j] * p1[c];
              for (int a = 0; a < 3; a++) g += mu[3 * j + a] * 2.0 * p2[a][c];
              for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) g += th[a][b] * 3.0 * p3[a][b][c];
              lg[c] -= q[i] * g; /* r depends on -R_mm */
            }
          }
    }
    for (int c = 0; c < 3; c++) agmm[4 * s + c] += lg[c];
    agmm[4 * s + 3] += lq;
  }

  /* ---------- 2. QM-QM real space, ordered pairs with 1/2 (main text, QM image energy) ---------- */
  if (P->qmqm) {
    for (int a = 0; a < nq; a++) {
      double tha[3][3];
      unpack_sym(theta + 6 * a, tha);
      for (int b = 0; b < nq; b++) {
        double thb[3][3];
        unpack_sym(theta + 6 * b, thb);
        for (int ix = -nix; ix <= nix; ix++)
          for (int iy = -niy; iy <= niy; iy++)
            for (int iz = -niz; iz <= niz; iz++) {
              if (a == b && ix == 0 && iy == 0 && iz == 0) continue;
              double r[3] = {qm_pos[3 * a + 0] - qm_pos[3 * b + 0] + ix * Lx,
                             qm_pos[3 * a + 1] - qm_pos[3 * b + 1] + iy * Ly,
                             qm_pos[3 * a + 2] - qm_pos[3 * b + 2] + iz * Lz};
              double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
              if (!(d2 < rc * rc)) continue;
              double p0, p1[3], p2[3][3], p3[3][3][3];
              real_tensors(r, al, &p0, p1, p2, p3);
              const double Qa = Q[a], Qb = Q[b];
              const double* ma = mu + 3 * a;
              const double* mb = mu + 3 * b;
              double Pv = Qa * Qb * p0;
              for (int c = 0; c < 3; c++) Pv += (Qb * ma[c] - Qa * mb[c]) * p1[c];
              for (int c = 0; c < 3; c++)
                for (int d = 0; d < 3; d++) {
                  Pv += (Qb * tha[c][d] + Qa * thb[c][d]) * p2[c][d];
                  Pv -= 2.0 * ma[c] * p2[c][d] * mb[d];
                }
              en[EN_QQ_SR] += 0.5L * Pv;
              /* gradient w.r.t. r (= R_a - R_b + image) */
              for (int g = 0; g < 3; g++) {
                double dg = Qa * Qb * p1[g];
                for (int c = 0; c < 3; c++) dg += (Qb * ma[c] - Qa * mb[c]) * 2.0 * p2[c][g];
                for (int c = 0; c < 3; c++)
                  for (int d = 0; d < 3; d++) {
                    dg += (Qb * tha[c][d] + Qa * thb[c][d]) * 3.0 * p3[c][d][g];
                    dg -= 2.0 * ma[c] * 3.0 * p3[c][d][g] * mb[d];
                  }
                agq[3 * a + g] += 0.5L * dg;
                agq[3 * b + g] -= 0.5L * dg;
              }
              /* moment derivatives (x 1/2 for ordered pairs) */
              {
                double dQa = Qb * p0, dQb = Qa * p0;
                for (int c = 0; c < 3; c++) {
                  dQa += -mb[c] * p1[c];
                  dQb += ma[c] * p1[c];
                }
                for (int c = 0; c < 3; c++)
                  for (int d = 0; d < 3; d++) {
                    dQa += thb[c][d] * p2[c][d];
                    dQb += tha[c][d] * p2[c][d];
                  }
                agm[10 * a + 0] += 0.5L * dQa;
                agm[10 * b + 0] += 0.5L * dQb;
                for (int c = 0; c < 3; c++) {
                  double dma = Qb * p1[c], dmb = -Qa * p1[c];
                  for (int d = 0; d < 3; d++) {
                    dma -= 2.0 * p2[c][d] * mb[d];
                    dmb -= 2.0 * ma[d] * p2[d][c];
                  }
                  agm[10 * a + 1 + c] += 0.5L * dma;
                  agm[10 * b + 1 + c] += 0.5L * dmb;
                }
                /* theta: derivative w.r.t. each distinct element of the full matrix;
                 * the stored-number multiplicity is applied at output time */
                for (int c = 0; c < 3; c++)
                  for (int d = c; d < 3; d++) {
                    agm[10 * a + 4 + sym6(c, d)] += 0.5L * Qb * p2[c][d];
                    agm[10 * b + 4 + sym6(c, d)] += 0.5L * Qa * p2[c][d];
                  }
              }
            }
      }
    }
  }

  /* ---------- 3. Reciprocal space (SI: point-charge and multipolar long-range terms) ---------- */
  const int nzl = 2 * mz + 1, nyl = 2 * my + 1, nxl = mx + 1;
  /* per-axis phase tables: tab[(atom*3 + axis)*(2m+1) + (n + m)] = e^{i 2 pi n x_axis / L_axis} */
  const int mmax = (mx > my ? (mx > mz ? mx : mz) : (my > mz ? my : mz));
  const int tw = 2 * mmax + 1;
  double* tq_re = malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1) * 3 * tw);
  double* tq_im = malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1) * 3 * tw);
  double* tm_re = malloc(sizeof(double) * (size_t)(nm > 0 ? nm : 1) * 3 * tw);
  double* tm_im = malloc(sizeof(double) * (size_t)(nm > 0 ? nm : 1) * 3 * tw);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nm; i++)
    for (int ax = 0; ax < 3; ax++)
      for (int n = -mmax; n <= mmax; n++) {
        double ang = 2.0 * PI * (double)n * mm_pos[3 * i + ax] / L[ax];
        tm_re[((size_t)i * 3 + ax) * tw + n + mmax] = cos(ang);
        tm_im[((size_t)i * 3 + ax) * tw + n + mmax] = sin(ang);
      }
  for (int j = 0; j < nq; j++)
    for (int ax = 0; ax < 3; ax++)
      for (int n = -mmax; n <= mmax; n++) {
        double ang = 2.0 * PI * (double)n * qm_pos[3 * j + ax] / L[ax];
        tq_re[((size_t)j * 3 + ax) * tw + n + mmax] = cos(ang);
        tq_im[((size_t)j * 3 + ax) * tw + n + mmax] = sin(ang);
      }
#define PH(tre, tim, atom, nx, ny, nz, outre, outim)                                           \
  do {                                                                                         \
    size_t bx_ = ((size_t)(atom) * 3 + 0) * tw + (nx) + mmax;                                  \
    size_t by_ = ((size_t)(atom) * 3 + 1) * tw + (ny) + mmax;                                  \
    size_t bz_ = ((size_t)(atom) * 3 + 2) * tw + (nz) + mmax;                                  \
    double xr_ = tre[bx_], xi_ = tim[bx_], yr_ = tre[by_], yi_ = tim[by_];                     \
    double xyr_ = xr_ * yr_ - xi_ * yi_, xyi_ = xr_ * yi_ + xi_ * yr_;                         \
    double zr_ = tre[bz_], zi_ = tim[bz_];                                                     \
    outre = xyr_ * zr_ - xyi_ * zi_;                                                           \
    outim = xyr_ * zi_ + xyi_ * zr_;                                                           \
  } while (0)

  /* k in the half space, flat index over the box [0..mx] x [-my..my] x [-mz..mz] */
  const size_t nk = (size_t)nxl * nyl * nzl;
  double* Smm = calloc(nk * 2, sizeof(double));  /* S_MM(k) */
  double* Sabc = calloc(nk * 6, sizeof(double)); /* A, B, C (re, im) */
  double* gk = calloc(nk, sizeof(double));       /* g(k) = e^{-k^2/4a^2}/k^2, 0 outside H */
  double* kv = calloc(nk * 3, sizeof(double));
  for (int nx = 0; nx <= mx; nx++)
    for (int ny = -my; ny <= my; ny++)
      for (int nz = -mz; nz <= mz; nz++) {
        size_t k = ((size_t)nx * nyl + (ny + my)) * nzl + (nz + mz);
        int inH = (nx > 0) || (nx == 0 && ny > 0) || (nx == 0 && ny == 0 && nz > 0);
        double kx = 2.0 * PI * nx / Lx, ky = 2.0 * PI * ny / Ly, kz = 2.0 * PI * nz / Lz;
        kv[3 * k + 0] = kx;
        kv[3 * k + 1] = ky;
        kv[3 * k + 2] = kz;
        double k2 = kx * kx + ky * ky + kz * kz;
        gk[k] = inH ? exp(-k2 / (4.0 * al * al)) / k2 : 0.0;
      }

  /* structure factors: S_MM(k) = sum_i q_i e^{i k.R_i}; A, B, C from the QM moments */
#pragma omp parallel for schedule(dynamic, 16)
  for (size_t k = 0; k < nk; k++) {
    if (gk[k] == 0.0) continue;
    int nz = (int)(k % nzl) - mz;
    int ny = (int)((k / nzl) % nyl) - my;
    int nx = (int)(k / ((size_t)nzl * nyl));
    long double sr = 0, si = 0;
    for (int i = 0; i < nm; i++) {
      double cr, ci;
      PH(tm_re, tm_im, i, nx, ny, nz, cr, ci);
      sr += q[i] * cr;
      si += q[i] * ci;
    }
    Smm[2 * k] = (double)sr;
    Smm[2 * k + 1] = (double)si;
    const double* kk = kv + 3 * k;
    long double ar = 0, ai = 0, br = 0, bi = 0, cr_ = 0, ci_ = 0;
    for (int j = 0; j < nq; j++) {
      double er, ei;
      PH(tq_re, tq_im, j, nx, ny, nz, er, ei);
      double th[3][3];
      unpack_sym(theta + 6 * j, th);
      double kmu = kk[0] * mu[3 * j] + kk[1] * mu[3 * j + 1] + kk[2] * mu[3 * j + 2];
      double kthk = 0.0;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) kthk += kk[a] * th[a][b] * kk[b];
      ar += Q[j] * er;
      ai += Q[j] * ei;
      /* i (k.mu) e */
      br += -kmu * ei;
      bi += kmu * er;
      /* -1/2 k.theta.k e */
      cr_ += -0.5 * kthk * er;
      ci_ += -0.5 * kthk * ei;
    }
    Sabc[6 * k + 0] = (double)ar;
    Sabc[6 * k + 1] = (double)ai;
    Sabc[6 * k + 2] = (double)br;
    Sabc[6 * k + 3] = (double)bi;
    Sabc[6 * k + 4] = (double)cr_;
    Sabc[6 * k + 5] = (double)ci_;
  }

  const double pref = 8.0 * PI / V; /* (4 pi / V) x 2 for the half space */

  /* energies from the structure factors */
  {
    long double eqm = 0, eqq = 0;
    for (size_t k = 0; k < nk; k++) {
      if (gk[k] == 0.0) continue;
      double ar = Sabc[6 * k], ai = Sabc[6 * k + 1], br = Sabc[6 * k + 2], bi = Sabc[6 * k + 3];
      double cr = Sabc[6 * k + 4], ci = Sabc[6 * k + 5];
      double sqr = ar + br + cr, sqi = ai + bi + ci;
      double smr = Smm[2 * k], smi = Smm[2 * k + 1];
      /* Re[S_QM conj(S_MM)] */
      eqm += pref * gk[k] * (sqr * smr + sqi * smi);
      /* |A|^2 + 2 Re(A* B) + 2 Re(A* C) + |B|^2 */
      double f = (ar * ar + ai * ai) + 2.0 * (ar * br + ai * bi) + 2.0 * (ar * cr + ai * ci) + (br * br + bi * bi);
      eqq += 0.5 * pref * gk[k] * f;
    }
    en[EN_QMMM_LR] = eqm;
    if (P->qmqm) en[EN_QQ_LR] = eqq;
  }

  /* QM-site projections: potential, field, half Hessian of the MM potential,
   * QM forces of the QM-MM and QM-QM terms, QM-QM moment derivatives */
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j < nq; j++) {
    double th[3][3];
    unpack_sym(theta + 6 * j, th);
    long double lp[10] = {0}, lg[3] = {0}, lm[10] = {0};
    for (size_t k = 0; k < nk; k++) {
      if (gk[k] == 0.0) continue;
      int nz = (int)(k % nzl) - mz;
      int ny = (int)((k / nzl) % nyl) - my;
      int nx = (int)(k / ((size_t)nzl * nyl));
      double er, ei;
      PH(tq_re, tq_im, j, nx, ny, nz, er, ei);
      const double* kk = kv + 3 * k;
      double w = pref * gk[k];
      /* Y = e^{i k.R_j} conj(S_MM) */
      double smr = Smm[2 * k], smi = Smm[2 * k + 1];
      double yr = er * smr + ei * smi, yi = ei * smr - er * smi;
      lp[0] += w * yr;
      for (int a = 0; a < 3; a++) lp[1 + a] += -w * kk[a] * yi;
      lp[4] += -0.5 * w * kk[0] * kk[0] * yr;
      lp[5] += -0.5 * w * kk[0] * kk[1] * yr;
      lp[6] += -0.5 * w * kk[0] * kk[2] * yr;
      lp[7] += -0.5 * w * kk[1] * kk[1] * yr;
      lp[8] += -0.5 * w * kk[1] * kk[2] * yr;
      lp[9] += -0.5 * w * kk[2] * kk[2] * yr;
      /* QM-MM force part: Re[i k_g w_j Y], w_j = Q + i k.mu - 1/2 k.theta.k */
      double kmu = kk[0] * mu[3 * j] + kk[1] * mu[3 * j + 1] + kk[2] * mu[3 * j + 2];
      double kthk = 0.0;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) kthk += kk[a] * th[a][b] * kk[b];
      double wr = Q[j] - 0.5 * kthk, wi = kmu;
      /* i (wr + i wi) (yr + i yi) = i(wr yr - wi yi) - (wr yi + wi yr) -> real part */
      double re_iwY = -(wr * yi + wi * yr);
      for (int g = 0; g < 3; g++) lg[g] += w * kk[g] * re_iwY;
      if (P->qmqm) {
        double ar = Sabc[6 * k], ai = Sabc[6 * k + 1], br = Sabc[6 * k + 2], bi = Sabc[6 * k + 3];
        double cr = Sabc[6 * k + 4], ci = Sabc[6 * k + 5];
        /* a_j = Q e, b_j = i kmu e, c_j = -1/2 kthk e */
        double ajr = Q[j] * er, aji = Q[j] * ei;
        double bjr = -kmu * ei, bji = kmu * er;
        double cjr = -0.5 * kthk * er, cji = -0.5 * kthk * ei;
        /* Z = a_j conj(A+B+C) + b_j conj(A+B) + c_j conj(A); only Im Z is needed */
        double t1r = ar + br + cr, t1i = ai + bi + ci;
        double t2r = ar + br, t2i = ai + bi;
        double zi = (aji * t1r - ajr * t1i) + (bji * t2r - bjr * t2i) + (cji * ar - cjr * ai);
        /* dE_QQ/dR_jg = (pref/2) g 2 Re[i k_g Z] = pref g k_g (-zi) */
        for (int g = 0; g < 3; g++) lg[g] += w * kk[g] * (-zi);
        /* dE_QQ/dQ_j = pref g Re[e conj(A+B+C)] */
        lm[0] += w * (er * t1r + ei * t1i);
        /* dE_QQ/dmu_j = pref g Re[i k e conj(A+B)] = pref g k (-(Im[e conj(A+B)])) */
        double im_e_t2 = ei * t2r - er * t2i;
        for (int a = 0; a < 3; a++) lm[1 + a] += -w * kk[a] * im_e_t2;
        /* dE_QQ/dtheta_ab (full) = pref g Re[-1/2 k_a k_b e conj(A)] */
        double re_e_a = er * ar + ei * ai;
        lm[4] += -0.5 * w * kk[0] * kk[0] * re_e_a;
        lm[5] += -0.5 * w * kk[0] * kk[1] * re_e_a;
        lm[6] += -0.5 * w * kk[0] * kk[2] * re_e_a;
        lm[7] += -0.5 * w * kk[1] * kk[1] * re_e_a;
        lm[8] += -0.5 * w * kk[1] * kk[2] * re_e_a;
        lm[9] += -0.5 * w * kk[2] * kk[2] * re_e_a;
      }
    }
    for (int t = 0; t < 10; t++) aphi[10 * j + t] += lp[t];
    for (int g = 0; g < 3; g++) agq[3 * j + g] += lg[g];
    for (int t = 0; t < 10; t++) agm[10 * j + t] += lm[t];
  }

  /* MM gradients: dE/dR_i = pref g q_i k Im[S_QM e^{-i k.R_i}], dE/dq_i = pref g Re[S_QM e^{-i k.R_i}] */
#pragma omp parallel for schedule(dynamic, 16)
  for (int s = 0; s < nsel; s++) {
    int i = (n_sel < 0) ? s : mm_sel[s];
    long double lg[3] = {0}, lq = 0;
    for (size_t k = 0; k < nk; k++) {
      if (gk[k] == 0.0) continue;
      int nz = (int)(k % nzl) - mz;
      int ny = (int)((k / nzl) % nyl) - my;
      int nx = (int)(k / ((size_t)nzl * nyl));
      double er, ei;
      PH(tm_re, tm_im, i, nx, ny, nz, er, ei);
      double sqr = Sabc[6 * k] + Sabc[6 * k + 2] + Sabc[6 * k + 4];
      double sqi = Sabc[6 * k + 1] + Sabc[6 * k + 3] + Sabc[6 * k + 5];
      /* S_QM conj(e) */
      double vr = sqr * er + sqi * ei, vi = sqi * er - sqr * ei;
      double w = pref * gk[k];
      const double* kk = kv + 3 * k;
      for (int g = 0; g < 3; g++) lg[g] += w * q[i] * kk[g] * vi;
      lq += w * vr;
    }
    for (int g = 0; g < 3; g++) agmm[4 * s + g] += lg[g];
    agmm[4 * s + 3] += lq;
  }

  /* ---------- 4. Self terms and neutralising background ---------- */
  const double bgc = P->background ? -PI / (al * al * V) : 0.0;
  if (P->qmqm) {
    long double es = 0;
    for (int j = 0; j < nq; j++) {
      const double* m = mu + 3 * j;
      const double* t = theta + 6 * j;
      double tr = t[0] + t[3] + t[5];
      double mm2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
      es += -al / sp * Q[j] * Q[j] - 2.0 * al * al * al / (3.0 * sp) * mm2 + 2.0 * al * al * al / (3.0 * sp) * Q[j] * tr;
      agm[10 * j + 0] += -2.0 * al / sp * Q[j] + 2.0 * al * al * al / (3.0 * sp) * tr + bgc * Qtot;
      for (int a = 0; a < 3; a++) agm[10 * j + 1 + a] += -4.0 * al * al * al / (3.0 * sp) * m[a];
      /* diagonal of theta (full matrix) */
      agm[10 * j + 4 + 0] += 2.0 * al * al * al / (3.0 * sp) * Q[j];
      agm[10 * j + 4 + 3] += 2.0 * al * al * al / (3.0 * sp) * Q[j];
      agm[10 * j + 4 + 5] += 2.0 * al * al * al / (3.0 * sp) * Q[j];
    }
    en[EN_QQ_SELF] = es;
    en[EN_QQ_BG] = 0.5 * bgc * Qtot * Qtot;
  }
  en[EN_QMMM_BG] = bgc * Qtot * qtot;
  for (int j = 0; j < nq; j++) aphi[10 * j + 0] += bgc * qtot;
  for (int s = 0; s < nsel; s++) agmm[4 * s + 3] += bgc * Qtot;

  /* ---------- 5. Outputs ---------- */
  long double etot = 0;
  for (int e = 1; e < EN_COUNT; e++) etot += en[e];
  if (energy) {
    energy[EN_TOTAL] = (double)etot;
    for (int e = 1; e < EN_COUNT; e++) energy[e] = (double)en[e];
  }
  for (int j = 0; j < nq; j++) {
    if (phi) phi[j] = (double)aphi[10 * j];
    if (dphi)
      for (int a = 0; a < 3; a++) dphi[3 * j + a] = (double)aphi[10 * j + 1 + a];
    if (hphi)
      for (int t = 0; t < 6; t++) hphi[6 * j + t] = (double)aphi[10 * j + 4 + t];
    if (g_qm_pos)
      for (int g = 0; g < 3; g++) g_qm_pos[3 * j + g] = (double)agq[3 * j + g];
    /* dE/dmoments = MM-generated field terms + QM-QM terms */
    if (g_Q) g_Q[j] = (double)(aphi[10 * j] + agm[10 * j]);
    if (g_mu)
      for (int a = 0; a < 3; a++) g_mu[3 * j + a] = (double)(aphi[10 * j + 1 + a] + agm[10 * j + 1 + a]);
    if (g_theta) {
      double full[3][3];
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) full[a][b] = (double)(aphi[10 * j + 4 + sym6(a, b)] + agm[10 * j + 4 + sym6(a, b)]);
      for (int t = 0; t < 6; t++) g_theta[6 * j + t] = 0.0;
      add_theta_grad(g_theta + 6 * j, full, 1.0);
    }
  }
  for (int s = 0; s < nsel; s++) {
    if (g_mm_pos)
      for (int g = 0; g < 3; g++) g_mm_pos[3 * s + g] = (double)agmm[4 * s + g];
    if (g_mm_q) g_mm_q[s] = (double)agmm[4 * s + 3];
  }

  free(wq);
  free(wm);
  free(aphi);
  free(agq);
  free(agm);
  free(agmm);
  free(tq_re);
  free(tq_im);
  free(tm_re);
  free(tm_im);
  free(Smm);
  free(Sabc);
  free(gk);
  free(kv);
  return 0;
}

/* OpenMP threads of later calls (timing only; no effect on the arithmetic's
 * definition, though the order of the per-thread partial sums follows it) */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ======================================================================
 * Region-I / region-II split (main text: periodic QM/MM multipole energy,
 * the Gaussian-charge correction; SI: bare tensors T, T_a, T_ab, T_abc and
 * the screened T-hat(kappa_i) with f1, f3, f5, f7).
 *
 * The Ewald sums above run over the whole lattice.  The quantities the SCF
 * consumes are those of region II only, obtained by subtracting the finite
 * direct sums over region I:
 *
 *   E_qq_bare = -1/2 sum_{a != b in QM} P_T(a, b)         unit-cell QM pairs,
 *               same pair form as the Ewald QM-QM term with bare tensors
 *   E_mm_bare = - sum_{(i,n) in MM(I)} sum_j q_i [Q_j T + mu_j.T_a + theta_j:T_ab]
 *   E_gauss   = - sum_{(i,n) in MM(II), kappa_i > 0, |r| < r_gauss} sum_j
 *                 q_i [Q_j That + mu_j.That_a + theta_j:That_ab]   (kappa = kappa_i)
 *
 * with r = R_j - (R_i + n L), C = arithmetic mean of the QM positions, and
 * MM(I) = { (i, n) : |R_i + n L - C| < r_region }, every lattice translate n
 * of every MM atom (the sphere may be larger than the cell), MM(II) its
 * complement.  The bare tensors are those of erfc(kappa r)/r at kappa = 0.
 * Readings frozen here: QM positions are used as passed (the QM subsystem
 * is one piece, QM-QM pair vectors and C are not wrapped); kappa_i <= 0 marks
 * a point charge, which has no Gaussian correction; r_gauss is one pair
 * cutoff for every Gaussian charge (the correction decays like erfc).
 *
 * Outputs (overwritten): energy[3] = {E_qq_bare, E_mm_bare, E_gauss};
 * phi, dphi, hphi: the correction to the MM potential, its gradient and
 * half Hessian at the QM sites (the MM(I) and Gaussian terms); g_*: the
 * gradient of E_qq_bare + E_mm_bare + E_gauss; counts[2] = {region-I images,
 * Gaussian (QM, MM image) pairs}.
 * ====================================================================== */
typedef struct {
  double box[3];
  double r_region;
  double r_gauss;
} oracle_region_t;

/* accumulate one (QM site j, MM image) pair with tensors of erfc(kappa r)/r,
 * scaled by s (= -1 for the subtractions) */
static void region_pair(const double r[3], double kappa, double s, double qi, double Qj, const double* mj,
                        double th[3][3], long double* phi10, long double* gq3, long double* gm4, long double* e) {
  double p0, p1[3], p2[3][3], p3[3][3][3];
  real_tensors(r, kappa, &p0, p1, p2, p3);
  phi10[0] += s * qi * p0;
  for (int a = 0; a < 3; a++) phi10[1 + a] += s * qi * p1[a];
  for (int a = 0; a < 3; a++)
    for (int b = a; b < 3; b++) phi10[4 + sym6(a, b)] += s * qi * p2[a][b];
  double en = Qj * p0;
  for (int a = 0; a < 3; a++) en += mj[a] * p1[a];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) en += th[a][b] * p2[a][b];
  *e += s * qi * en;
  for (int c = 0; c < 3; c++) {
    double g = Qj * p1[c];
    for (int a = 0; a < 3; a++) g += mj[a] * 2.0 * p2[a][c];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) g += th[a][b] * 3.0 * p3[a][b][c];
    gq3[c] += s * qi * g;   /* d/dR_j */
    gm4[c] -= s * qi * g;   /* d/dR_i: r depends on -R_i */
  }
  gm4[3] += s * en;         /* d/dq_i */
}

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

int oracle_region(const oracle_region_t* P, int nq, const double* qm_pos, const double* Q, const double* mu,
                  const double* theta, int nm, const double* mm_pos, const double* q, const double* kappa,
                  double* energy, double* phi, double* dphi, double* hphi, double* g_qm_pos, double* g_Q,
                  double* g_mu, double* g_theta, double* g_mm_pos, double* g_mm_q, long* counts) {
  const double* L = P->box;
  if (nq < 0 || nm < 0 || L[0] <= 0.0 || L[1] <= 0.0 || L[2] <= 0.0 || P->r_region < 0.0 || P->r_gauss < 0.0)
    return -1;
  const double R1 = P->r_region, RG = P->r_gauss;
  double C[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < nq; j++)
    for (int a = 0; a < 3; a++) C[a] += qm_pos[3 * j + a];
  for (int a = 0; a < 3; a++) C[a] = nq > 0 ? C[a] / nq : 0.0;

  long double* aphi = calloc((size_t)(nq > 0 ? nq : 1) * 10, sizeof(long double));
  long double* agq = calloc((size_t)(nq > 0 ? nq : 1) * 3, sizeof(long double));
  long double* agm = calloc((size_t)(nq > 0 ? nq : 1) * 10, sizeof(long double));
  long double* agmm = calloc((size_t)(nm > 0 ? nm : 1) * 4, sizeof(long double));
  long double e_qq = 0.0L, e_mm = 0.0L, e_g = 0.0L;
  long n_img = 0, n_gp = 0;

  /* 1. MM(I) and the Gaussian correction, one MM atom at a time */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : n_img, n_gp)
  for (int i = 0; i < nm; i++) {
    const double* Ri = mm_pos + 3 * i;
    long double lgm[4] = {0, 0, 0, 0}, lemm = 0.0L, leg = 0.0L;
    long double* lphi = calloc((size_t)(nq > 0 ? nq : 1) * 10, sizeof(long double));
    long double* lgq = calloc((size_t)(nq > 0 ? nq : 1) * 3, sizeof(long double));
    /* every lattice translate within r_region of C: a generous box of n, then the test */
    int N[3];
    for (int a = 0; a < 3; a++) N[a] = (int)ceil((R1 + fabs(Ri[a] - C[a])) / L[a]) + 1;
    for (int nx = -N[0]; nx <= N[0]; nx++)
      for (int ny = -N[1]; ny <= N[1]; ny++)
        for (int nz = -N[2]; nz <= N[2]; nz++) {
          double Ri_n[3] = {Ri[0] + nx * L[0], Ri[1] + ny * L[1], Ri[2] + nz * L[2]};
          double dC[3] = {Ri_n[0] - C[0], Ri_n[1] - C[1], Ri_n[2] - C[2]};
          if (!(norm3(dC) < R1)) continue;
          n_img++;
          for (int j = 0; j < nq; j++) {
            double th[3][3];
            unpack_sym(theta + 6 * j, th);
            double r[3] = {qm_pos[3 * j] - Ri_n[0], qm_pos[3 * j + 1] - Ri_n[1], qm_pos[3 * j + 2] - Ri_n[2]};
            region_pair(r, 0.0, -1.0, q[i], Q[j], mu + 3 * j, th, lphi + 10 * j, lgq + 3 * j, lgm, &lemm);
          }
        }
    /* Gaussian charges: region-II translates within r_gauss of a QM site */
    if (kappa && kappa[i] > 0.0) {
      for (int j = 0; j < nq; j++) {
        double th[3][3];
        unpack_sym(theta + 6 * j, th);
        const double* Rj = qm_pos + 3 * j;
        int M[3];
        for (int a = 0; a < 3; a++) M[a] = (int)ceil((RG + fabs(Rj[a] - Ri[a])) / L[a]) + 1;
        for (int nx = -M[0]; nx <= M[0]; nx++)
          for (int ny = -M[1]; ny <= M[1]; ny++)
            for (int nz = -M[2]; nz <= M[2]; nz++) {
              double Ri_n[3] = {Ri[0] + nx * L[0], Ri[1] + ny * L[1], Ri[2] + nz * L[2]};
              double dC[3] = {Ri_n[0] - C[0], Ri_n[1] - C[1], Ri_n[2] - C[2]};
              if (norm3(dC) < R1) continue; /* region I: already direct */
              double r[3] = {Rj[0] - Ri_n[0], Rj[1] - Ri_n[1], Rj[2] - Ri_n[2]};
              if (!(norm3(r) < RG)) continue;
              n_gp++;
              region_pair(r, kappa[i], -1.0, q[i], Q[j], mu + 3 * j, th, lphi + 10 * j, lgq + 3 * j, lgm, &leg);
            }
      }
    }
    for (int t = 0; t < 4; t++) agmm[4 * i + t] += lgm[t];
#pragma omp critical
    {
      for (int t = 0; t < 10 * nq; t++) aphi[t] += lphi[t];
      for (int t = 0; t < 3 * nq; t++) agq[t] += lgq[t];
      e_mm += lemm;
      e_g += leg;
    }
    free(lphi);
    free(lgq);
  }

  /* 2. unit-cell QM-QM pairs with bare tensors: -1/2 sum over ordered pairs a != b */
  for (int a = 0; a < nq; a++) {
    double tha[3][3];
    unpack_sym(theta + 6 * a, tha);
    for (int b = 0; b < nq; b++) {
      if (a == b) continue;
      double thb[3][3];
      unpack_sym(theta + 6 * b, thb);
      double r[3] = {qm_pos[3 * a] - qm_pos[3 * b], qm_pos[3 * a + 1] - qm_pos[3 * b + 1],
                     qm_pos[3 * a + 2] - qm_pos[3 * b + 2]};
      double p0, p1[3], p2[3][3], p3[3][3][3];
      real_tensors(r, 0.0, &p0, p1, p2, p3);
      const double Qa = Q[a], Qb = Q[b];
      const double* ma = mu + 3 * a;
      const double* mb = mu + 3 * b;
      double Pv = Qa * Qb * p0;
      for (int c = 0; c < 3; c++) Pv += (Qb * ma[c] - Qa * mb[c]) * p1[c];
      for (int c = 0; c < 3; c++)
        for (int d = 0; d < 3; d++) {
          Pv += (Qb * tha[c][d] + Qa * thb[c][d]) * p2[c][d];
          Pv -= 2.0 * ma[c] * p2[c][d] * mb[d];
        }
      e_qq += -0.5L * Pv;
      for (int g = 0; g < 3; g++) {
        double dg = Qa * Qb * p1[g];
        for (int c = 0; c < 3; c++) dg += (Qb * ma[c] - Qa * mb[c]) * 2.0 * p2[c][g];
        for (int c = 0; c < 3; c++)
          for (int d = 0; d < 3; d++) {
            dg += (Qb * tha[c][d] + Qa * thb[c][d]) * 3.0 * p3[c][d][g];
            dg -= 2.0 * ma[c] * 3.0 * p3[c][d][g] * mb[d];
          }
        agq[3 * a + g] += -0.5L * dg;
        agq[3 * b + g] -= -0.5L * dg;
      }
      double dQa = Qb * p0, dQb = Qa * p0;
      for (int c = 0; c < 3; c++) {
        dQa += -mb[c] * p1[c];
        dQb += ma[c] * p1[c];
      }
      for (int c = 0; c < 3; c++)
        for (int d = 0; d < 3; d++) {
          dQa += thb[c][d] * p2[c][d];
          dQb += tha[c][d] * p2[c][d];
        }
      agm[10 * a] += -0.5L * dQa;
      agm[10 * b] += -0.5L * dQb;
      for (int c = 0; c < 3; c++) {
        double dma = Qb * p1[c], dmb = -Qa * p1[c];
        for (int d = 0; d < 3; d++) {
          dma -= 2.0 * p2[c][d] * mb[d];
          dmb -= 2.0 * ma[d] * p2[d][c];
        }
        agm[10 * a + 1 + c] += -0.5L * dma;
        agm[10 * b + 1 + c] += -0.5L * dmb;
      }
      /* full-matrix theta derivatives, stored by sym6 index (each element of
       * the symmetric pair is visited, so off-diagonals collect both) */
      for (int c = 0; c < 3; c++)
        for (int d = 0; d < 3; d++) {
          agm[10 * a + 4 + sym6(c, d)] += -0.5L * Qb * p2[c][d];
          agm[10 * b + 4 + sym6(c, d)] += -0.5L * Qa * p2[c][d];
        }
    }
  }

  /* 3. outputs */
  if (energy) {
    energy[0] = (double)e_qq;
    energy[1] = (double)e_mm;
    energy[2] = (double)e_g;
  }
  for (int j = 0; j < nq; j++) {
    if (phi) phi[j] = (double)aphi[10 * j];
    if (dphi)
      for (int a = 0; a < 3; a++) dphi[3 * j + a] = (double)aphi[10 * j + 1 + a];
    if (hphi)
      for (int t = 0; t < 6; t++) hphi[6 * j + t] = (double)aphi[10 * j + 4 + t];
    if (g_qm_pos)
      for (int g = 0; g < 3; g++) g_qm_pos[3 * j + g] = (double)agq[3 * j + g];
    if (g_Q) g_Q[j] = (double)(aphi[10 * j] + agm[10 * j]);
    if (g_mu)
      for (int a = 0; a < 3; a++) g_mu[3 * j + a] = (double)(aphi[10 * j + 1 + a] + agm[10 * j + 1 + a]);
    if (g_theta) {
      /* MM field part: dE/dtheta_ab (full) = half Hessian; stored numbers take
       * both off-diagonal elements.  QM-QM part is already per stored number. */
      double full[3][3];
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) full[a][b] = (double)aphi[10 * j + 4 + sym6(a, b)];
      for (int t = 0; t < 6; t++) g_theta[6 * j + t] = (double)agm[10 * j + 4 + t];
      add_theta_grad(g_theta + 6 * j, full, 1.0);
    }
  }
  for (int i = 0; i < nm; i++) {
    if (g_mm_pos)
      for (int g = 0; g < 3; g++) g_mm_pos[3 * i + g] = (double)agmm[4 * i + g];
    if (g_mm_q) g_mm_q[i] = (double)agmm[4 * i + 3];
  }
  if (counts) {
    counts[0] = n_img;
    counts[1] = n_gp;
  }
  free(aphi);
  free(agq);
  free(agm);
  free(agmm);
  return 0;
}

/* ======================================================================
 * Charge-octupole error estimate (main text, Error Control: the leading
 * error of the quadrupole-truncated expansion is the interaction of the
 * region-II charges with the QM octupoles; SI: T_abc = 1/3 d/dR_c T_ab).
 *
 *   Err(R_cut) = sum_{(i,n): R_cut <= |R_i + n L - C| < r_outer} sum_j
 *                q_i sum_{abc} Omega_j,abc T_abc(R_j - R_i - n L)
 *   T_abc(r) = -[5 r_a r_b r_c - r^2 (r_a d_bc + r_b d_ac + r_c d_ab)] / (2 r^7)
 *
 * Omega_j is the raw (not traceless) third moment of site j, stored as its
 * ten distinct components xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz.
 * Readings frozen here: the site index of the octupole is the QM site j (the
 * printed formula carries the MM index on Omega); the region-II sum, which
 * converges absolutely, is truncated at the outer radius r_outer around C;
 * the same centre C and translate rule as oracle_region.  Every candidate
 * R_cut is summed from scratch.
 * ====================================================================== */
static int oct_index(int a, int b, int c) {
  /* sort the three indices, then position in xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz */
  int s[3] = {a, b, c};
  for (int i = 0; i < 2; i++)
    for (int k = 0; k < 2 - i; k++)
      if (s[k] > s[k + 1]) {
        int t = s[k];
        s[k] = s[k + 1];
        s[k + 1] = t;
      }
  static const int table[3][3][3] = {
      {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}},
      {{1, 3, 4}, {3, 6, 7}, {4, 7, 8}},
      {{2, 4, 5}, {4, 7, 8}, {5, 8, 9}}};
  return table[s[0]][s[1]][s[2]];
}

int oracle_octupole_error(const double box[3], int nq, const double* qm_pos, const double* omega, int nm,
                          const double* mm_pos, const double* q, int n_r, const double* r_cut, double r_outer,
                          double* err) {
  if (nq < 0 || nm < 0 || n_r < 0 || box[0] <= 0.0 || box[1] <= 0.0 || box[2] <= 0.0 || r_outer < 0.0) return -1;
  double C[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < nq; j++)
    for (int a = 0; a < 3; a++) C[a] += qm_pos[3 * j + a];
  for (int a = 0; a < 3; a++) C[a] = nq > 0 ? C[a] / nq : 0.0;
  for (int k = 0; k < n_r; k++) {
    long double s = 0.0L;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : s)
    for (int i = 0; i < nm; i++) {
      const double* Ri = mm_pos + 3 * i;
      int N[3];
      for (int a = 0; a < 3; a++) N[a] = (int)ceil((r_outer + fabs(Ri[a] - C[a])) / box[a]) + 1;
      for (int nx = -N[0]; nx <= N[0]; nx++)
        for (int ny = -N[1]; ny <= N[1]; ny++)
          for (int nz = -N[2]; nz <= N[2]; nz++) {
            double Ri_n[3] = {Ri[0] + nx * box[0], Ri[1] + ny * box[1], Ri[2] + nz * box[2]};
            double dC[3] = {Ri_n[0] - C[0], Ri_n[1] - C[1], Ri_n[2] - C[2]};
            double D = norm3(dC);
            if (!(D >= r_cut[k] && D < r_outer)) continue;
            for (int j = 0; j < nq; j++) {
              double r[3] = {qm_pos[3 * j] - Ri_n[0], qm_pos[3 * j + 1] - Ri_n[1], qm_pos[3 * j + 2] - Ri_n[2]};
              double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
              double r7 = r2 * r2 * r2 * sqrt(r2);
              double e = 0.0;
              for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                  for (int c = 0; c < 3; c++) {
                    double dd = 0.0;
                    if (b == c) dd += r[a];
                    if (a == c) dd += r[b];
                    if (a == b) dd += r[c];
                    double T = -(5.0 * r[a] * r[b] * r[c] - r2 * dd) / (2.0 * r7);
                    e += omega[10 * j + oct_index(a, b, c)] * T;
                  }
              s += q[i] * e;
            }
          }
    }
    err[k] = (double)s;
  }
  return 0;
}

/* The smallest candidate whose estimate and the next candidate's are both
 * below eps in magnitude (main text: R_cut is raised in fixed steps from a
 * lower bound until two consecutive values pass); -1 if no such pair. */
double oracle_rcut_pick(int n_r, const double* r_cut, const double* err, double eps) {
  for (int k = 0; k + 1 < n_r; k++)
    if (fabs(err[k]) < eps && fabs(err[k + 1]) < eps) return r_cut[k];
  return -1.0;
}
