/*
 * A plain C program that uses the library only through include/mpewald.h and
 * the HIP runtime (no Python): one small periodic system through
 * ewald_forward (with the saved context), ewald_backward with unit upstream
 * gradient, ewald_region_forward/backward and ewald_octupole_error, each
 * result compared with the CPU oracle (linked from oracle/ewald_oracle.c; test
 * infrastructure only).  Exit status 0 when every relative error is within
 * 1e-10 and the error paths return their documented status codes.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/mpewald.h"

/* the oracle's entry points (oracle/ewald_oracle.c) */
typedef struct {
  double box[3];
  double alpha;
  double rcut;
  int kmax[3];
  int qmqm;
  int background;
} oracle_params_t;
typedef struct {
  double box[3];
  double r_region;
  double r_gauss;
} oracle_region_t;
int oracle_ewald(const oracle_params_t* P, int nq, const double* qm_pos, const double* Q, const double* mu,
                 const double* theta, int nm, const double* mm_pos, const double* q, double* energy, double* phi,
                 double* dphi, double* hphi, double* g_qm_pos, double* g_Q, double* g_mu, double* g_theta, int n_sel,
                 const int* mm_sel, double* g_mm_pos, double* g_mm_q);
int oracle_region(const oracle_region_t* P, int nq, const double* qm_pos, const double* Q, const double* mu,
                  const double* theta, int nm, const double* mm_pos, const double* q, const double* kappa,
                  double* energy, double* phi, double* dphi, double* hphi, double* g_qm_pos, double* g_Q,
                  double* g_mu, double* g_theta, double* g_mm_pos, double* g_mm_q, long* counts);
int oracle_octupole_error(const double box[3], int nq, const double* qm_pos, const double* omega, int nm,
                          const double* mm_pos, const double* q, int n_r, const double* r_cut, double r_outer,
                          double* err);
double oracle_rcut_pick(int n_r, const double* r_cut, const double* err, double eps);

#define NQ 7
#define NM 900
#define NR 6

static unsigned long long rng_state = 0x2408032730ull;
static double rnd(void) { /* 64-bit LCG, top 53 bits */
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(rng_state >> 11) / 9007199254740992.0;
}

static double relerr(const double* a, const double* b, int n) {
  double num = 0.0, den = 0.0;
  for (int i = 0; i < n; i++) {
    num = fmax(num, fabs(a[i] - b[i]));
    den = fmax(den, fabs(b[i]));
  }
  return den > 0.0 ? num / den : num;
}

static int failures = 0;
static void check(const char* what, double err, double tol) {
  printf("%-28s %.2e %s\n", what, err, err <= tol ? "ok" : "FAIL");
  if (!(err <= tol)) failures++;
}

#define HIPOK(x)                                                     \
  do {                                                               \
    if ((x) != hipSuccess) {                                         \
      fprintf(stderr, "HIP call failed: %s\n", #x);                  \
      return 2;                                                      \
    }                                                                \
  } while (0)

/* device copy of n doubles (h == NULL: allocation only) */
static double* dev_copy(const double* h, size_t n) {
  double* d = NULL;
  if (hipMalloc((void**)&d, (n ? n : 1) * sizeof(double)) != hipSuccess) return NULL;
  if (h && n && hipMemcpy(d, h, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return NULL;
  return d;
}

static int host_copy(double* h, const double* d, size_t n) {
  return hipMemcpy(h, d, n * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess ? 0 : 1;
}

int main(void) {
  const double box[3] = {17.0, 18.0, 19.0};
  static double qm[3 * NQ], Q[NQ], mu[3 * NQ], th[6 * NQ], mm[3 * NM], q[NM], kap[NM], om[10 * NQ];
  for (int j = 0; j < NQ; j++) {
    for (int a = 0; a < 3; a++) qm[3 * j + a] = box[a] * (0.4 + 0.2 * rnd());
    Q[j] = 1.8 * rnd() - 0.9;
    for (int a = 0; a < 3; a++) mu[3 * j + a] = 0.3 * (rnd() - 0.5);
    for (int a = 0; a < 6; a++) th[6 * j + a] = 0.2 * (rnd() - 0.5);
    for (int a = 0; a < 10; a++) om[10 * j + a] = 0.1 * (rnd() - 0.5);
  }
  for (int i = 0; i < NM; i++) {
    for (int a = 0; a < 3; a++) mm[3 * i + a] = box[a] * rnd();
    q[i] = 1.8 * rnd() - 0.9;
    kap[i] = (i % 3 == 0) ? 0.0 : 0.4 + 0.4 * rnd();
  }

  /* ---- library ---- */
  ewald_params_t p;
  memset(&p, 0, sizeof(p));
  for (int a = 0; a < 3; a++) p.box[a] = box[a];
  p.alpha = 0.38;
  p.rcut = 8.0;
  p.kmax[0] = 7;
  p.kmax[1] = 8;
  p.kmax[2] = 9;
  p.precision = EWALD_FP64;
  p.flags = EWALD_QMQM | EWALD_CELL_LIST;
  p.max_qm = NQ;
  p.max_mm = NM;
  p.max_frames = 1;
  ewald_plan* plan = NULL;
  if (ewald_setup(&p, &plan) != EWALD_OK) {
    fprintf(stderr, "ewald_setup: %s\n", ewald_last_error());
    return 2;
  }
  double *d_qm = dev_copy(qm, 3 * NQ), *d_Q = dev_copy(Q, NQ), *d_mu = dev_copy(mu, 3 * NQ),
         *d_th = dev_copy(th, 6 * NQ), *d_mm = dev_copy(mm, 3 * NM), *d_q = dev_copy(q, NM),
         *d_kap = dev_copy(kap, NM), *d_om = dev_copy(om, 10 * NQ);
  double* d_out = dev_copy(NULL, 1 + 10 * NQ + 13 * NQ + 4 * NM + NR + 1);
  if (!d_qm || !d_Q || !d_mu || !d_th || !d_mm || !d_q || !d_kap || !d_om || !d_out) return 2;
  double *d_E = d_out, *d_phi = d_E + 1, *d_ef = d_phi + NQ, *d_eg = d_ef + 3 * NQ;
  double *d_gq = d_eg + 6 * NQ, *d_gQ = d_gq + 3 * NQ, *d_gmu = d_gQ + NQ, *d_gth = d_gmu + 3 * NQ;
  double *d_gm = d_gth + 6 * NQ, *d_gmq = d_gm + 3 * NM, *d_err = d_gmq + NM, *d_rc = d_err + NR;
  void* ctx = NULL;
  HIPOK(hipMalloc(&ctx, ewald_ctx_bytes(plan, NQ, NM)));
  hipStream_t s;
  HIPOK(hipStreamCreate(&s));

  if (ewald_forward(plan, NQ, d_qm, d_Q, d_mu, d_th, NM, d_mm, d_q, d_E, d_phi, d_ef, d_eg, ctx, s) != EWALD_OK ||
      ewald_backward(plan, ctx, NQ, d_qm, d_Q, d_mu, d_th, NM, d_mm, d_q, NULL, NULL, NULL, NULL, d_gq, d_gQ, d_gmu,
                     d_gth, d_gm, d_gmq, s) != EWALD_OK) {
    fprintf(stderr, "ewald_forward/backward: %s\n", ewald_last_error());
    return 2;
  }
  HIPOK(hipStreamSynchronize(s));
  static double E[1], phi[NQ], ef[3 * NQ], eg[6 * NQ], gq[3 * NQ], gQ[NQ], gmu[3 * NQ], gth[6 * NQ], gm[3 * NM],
      gmq[NM];
  if (host_copy(E, d_E, 1) || host_copy(phi, d_phi, NQ) || host_copy(ef, d_ef, 3 * NQ) ||
      host_copy(eg, d_eg, 6 * NQ) || host_copy(gq, d_gq, 3 * NQ) || host_copy(gQ, d_gQ, NQ) ||
      host_copy(gmu, d_gmu, 3 * NQ) || host_copy(gth, d_gth, 6 * NQ) || host_copy(gm, d_gm, 3 * NM) ||
      host_copy(gmq, d_gmq, NM))
    return 2;

  /* ---- oracle ---- */
  oracle_params_t op;
  for (int a = 0; a < 3; a++) op.box[a] = box[a];
  op.alpha = p.alpha;
  op.rcut = p.rcut;
  for (int a = 0; a < 3; a++) op.kmax[a] = p.kmax[a];
  op.qmqm = 1;
  op.background = 1;
  static double oE[8], ophi[NQ], odphi[3 * NQ], ohphi[6 * NQ], ogq[3 * NQ], ogQ[NQ], ogmu[3 * NQ], ogth[6 * NQ],
      ogm[3 * NM], ogmq[NM], oef[3 * NQ], oeg[6 * NQ];
  if (oracle_ewald(&op, NQ, qm, Q, mu, th, NM, mm, q, oE, ophi, odphi, ohphi, ogq, ogQ, ogmu, ogth, -1, NULL, ogm,
                   ogmq) != 0)
    return 2;
  for (int t = 0; t < 3 * NQ; t++) oef[t] = -odphi[t];
  for (int t = 0; t < 6 * NQ; t++) oeg[t] = -2.0 * ohphi[t];
  check("energy", relerr(E, oE, 1), 1e-10);
  check("phi", relerr(phi, ophi, NQ), 1e-10);
  check("efield", relerr(ef, oef, 3 * NQ), 1e-10);
  check("efgrad", relerr(eg, oeg, 6 * NQ), 1e-10);
  check("g_qm_xyz", relerr(gq, ogq, 3 * NQ), 1e-10);
  check("g_Q", relerr(gQ, ogQ, NQ), 1e-10);
  check("g_mu", relerr(gmu, ogmu, 3 * NQ), 1e-10);
  check("g_theta", relerr(gth, ogth, 6 * NQ), 1e-10);
  check("g_mm_xyz", relerr(gm, ogm, 3 * NM), 1e-10);
  check("g_mm_q", relerr(gmq, ogmq, NM), 1e-10);

  /* ---- region split, added on top of the Ewald outputs ---- */
  const double rr = 6.5, rg = 9.0; /* r_gauss above half the box: all translates within it */
  if (ewald_region_forward(plan, NQ, d_qm, d_Q, d_mu, d_th, NM, d_mm, d_q, d_kap, rr, rg, d_E, d_phi, d_ef, d_eg,
                           s) != EWALD_OK ||
      ewald_region_backward(plan, NQ, d_qm, d_Q, d_mu, d_th, NM, d_mm, d_q, d_kap, rr, rg, NULL, NULL, NULL, NULL,
                            d_gq, d_gQ, d_gmu, d_gth, d_gm, d_gmq, s) != EWALD_OK) {
    fprintf(stderr, "ewald_region_*: %s\n", ewald_last_error());
    return 2;
  }
  HIPOK(hipStreamSynchronize(s));
  if (host_copy(E, d_E, 1) || host_copy(phi, d_phi, NQ) || host_copy(gq, d_gq, 3 * NQ) ||
      host_copy(gth, d_gth, 6 * NQ) || host_copy(gm, d_gm, 3 * NM) || host_copy(gmq, d_gmq, NM))
    return 2;
  oracle_region_t orp = {{box[0], box[1], box[2]}, rr, rg};
  static double rE[3], rphi[NQ], rdphi[3 * NQ], rhphi[6 * NQ], rgq[3 * NQ], rgQ[NQ], rgmu[3 * NQ], rgth[6 * NQ],
      rgm[3 * NM], rgmq[NM];
  long counts[2];
  if (oracle_region(&orp, NQ, qm, Q, mu, th, NM, mm, q, kap, rE, rphi, rdphi, rhphi, rgq, rgQ, rgmu, rgth, rgm, rgmq,
                    counts) != 0)
    return 2;
  double tE = oE[0] + rE[0] + rE[1] + rE[2];
  for (int t = 0; t < NQ; t++) rphi[t] += ophi[t];
  for (int t = 0; t < 3 * NQ; t++) rgq[t] += ogq[t];
  for (int t = 0; t < 6 * NQ; t++) rgth[t] += ogth[t];
  for (int t = 0; t < 3 * NM; t++) rgm[t] += ogm[t];
  for (int t = 0; t < NM; t++) rgmq[t] += ogmq[t];
  printf("region I translates %ld, Gaussian pairs %ld\n", counts[0], counts[1]);
  check("region energy", relerr(E, &tE, 1), 1e-10);
  check("region phi", relerr(phi, rphi, NQ), 1e-10);
  check("region g_qm_xyz", relerr(gq, rgq, 3 * NQ), 1e-10);
  check("region g_theta", relerr(gth, rgth, 6 * NQ), 1e-10);
  check("region g_mm_xyz", relerr(gm, rgm, 3 * NM), 1e-10);
  check("region g_mm_q", relerr(gmq, rgmq, NM), 1e-10);

  /* ---- octupole estimate and R_cut pick ---- */
  double cands[NR], oerr[NR], err[NR], rc;
  for (int k = 0; k < NR; k++) cands[k] = 3.0 + 1.5 * (double)k;
  if (oracle_octupole_error(box, NQ, qm, om, NM, mm, q, NR, cands, 15.0, oerr) != 0) return 2;
  const double eps = 0.5 * (fabs(oerr[2]) + fabs(oerr[3]));
  if (ewald_octupole_error(plan, NQ, d_qm, d_om, NM, d_mm, d_q, NR, 3.0, 1.5, 15.0, eps, d_err, d_rc, s) != EWALD_OK) {
    fprintf(stderr, "ewald_octupole_error: %s\n", ewald_last_error());
    return 2;
  }
  HIPOK(hipStreamSynchronize(s));
  if (host_copy(err, d_err, NR) || host_copy(&rc, d_rc, 1)) return 2;
  check("octupole estimate", relerr(err, oerr, NR), 1e-10);
  const double orc = oracle_rcut_pick(NR, cands, oerr, eps);
  check("R_cut pick", fabs(rc - orc), 0.0);

  /* ---- documented error paths: status code, message, nothing enqueued ---- */
  check("null plan -> ERR_ARG",
        ewald_forward(NULL, NQ, d_qm, d_Q, d_mu, d_th, NM, d_mm, d_q, d_E, NULL, NULL, NULL, NULL, s) ==
                EWALD_ERR_ARG && ewald_last_error()[0] != '\0'
            ? 0.0
            : 1.0,
        0.0);
  check("capacity -> ERR_CAPACITY",
        ewald_forward(plan, NQ + 1, d_qm, d_Q, d_mu, d_th, NM, d_mm, d_q, d_E, NULL, NULL, NULL, NULL, s) ==
                EWALD_ERR_CAPACITY
            ? 0.0
            : 1.0,
        0.0);
  check("region radius -> ERR_CUTOFF",
        ewald_region_forward(plan, NQ, d_qm, d_Q, d_mu, d_th, NM, d_mm, d_q, d_kap, 100.0, 0.0, d_E, NULL, NULL,
                             NULL, s) == EWALD_ERR_CUTOFF
            ? 0.0
            : 1.0,
        0.0);

  (void)hipStreamDestroy(s);
  (void)hipFree(ctx);
  ewald_destroy(plan);
  printf(failures ? "FAILED (%d)\n" : "all checks passed\n", failures);
  return failures ? 1 : 0;
}
