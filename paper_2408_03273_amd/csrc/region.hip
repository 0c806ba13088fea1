// Region-I / region-II split of the periodic multipole coupling on gfx950.
//
// Paper: Methods, the periodic QM/MM multipole energy written as whole-lattice
// Ewald sums minus direct sums over region I (a sphere of radius R_cut around
// the geometric centre of the QM atoms), and the correction for Gaussian-
// smeared MM charges in region II; Supporting Information, the bare tensors
// T, T_a, T_ab, T_abc and the screened ones with f1, f3, f5, f7 at kappa_i.
//
// The terms added to the Ewald outputs are
//   - the bare QM-QM pairs of the unit cell, -1/2 sum_{a != b} P_T(a, b);
//   - the bare interaction with every MM lattice translate inside the sphere;
//   - the erfc(kappa_i r)/r interaction with every region-II translate of a
//     Gaussian MM charge (kappa_i > 0) within r_gauss of a QM site,
// each with a minus sign.  These are finite real-space sums over at most a
// few thousand MM translates per QM site: plain FP64 VALU pair kernels over
// (QM site, MM chunk) blocks that skip the MM atoms a preparation pass has not
// flagged, and one wave per group of 64 MM atoms for the MM gradients.
#include <math.h>

#include <algorithm>

#include "ewald_internal.h"

namespace mpe {

#define DEV __device__ __forceinline__

struct RadialK {
  double f1, f3, f5, f7;
};

// Radial functions of erfc(kappa r)/r (SI: f1, f3, f5, f7); kappa = 0 gives
// the bare 1/r^(2n+1).
DEV RadialK radial_k(double r2, double kappa) {
  const double r = sqrt(r2);
  const double inv2 = 1.0 / r2;
  RadialK o;
  if (kappa > 0.0) {
    const double ex = exp(-kappa * kappa * r2);
    const double c = 1.1283791670955126 * kappa;  // 2 kappa / sqrt(pi)
    o.f1 = erfc(kappa * r) / r;
    o.f3 = (o.f1 + c * ex) * inv2;
    o.f5 = (o.f3 + (2.0 / 3.0) * kappa * kappa * c * ex) * inv2;
    o.f7 = (o.f5 + (4.0 / 15.0) * kappa * kappa * kappa * kappa * c * ex) * inv2;
  } else {
    o.f1 = 1.0 / r;
    o.f3 = o.f1 * inv2;
    o.f5 = o.f3 * inv2;
    o.f7 = o.f5 * inv2;
  }
  return o;
}

// Moments of one site as the pair kernels use them: Q, mu, theta (full
// symmetric, stored order xx,xy,xz,yy,yz,zz).
struct Site {
  double Q, m[3], t[6];
};

// Effective moments of the adjoint: L = gE E + g_phi.phi + g_efield.efield +
// g_efgrad.efgrad is, site by site, the energy of the moments
// (gE Q + g_phi, gE mu - g_efield, gE theta - w g_efgrad), w = 2 on the
// diagonal and 1 off it (efgrad = -2 x half Hessian, off-diagonal stored
// numbers count twice in theta : H).
DEV Site eff_site(const RegionArgs& ra, int j, double gE, const double* g_phi, const double* g_efield,
                  const double* g_efgrad) {
  Site s;
  s.Q = gE * ra.Q[j] + (g_phi ? g_phi[j] : 0.0);
  for (int a = 0; a < 3; a++) s.m[a] = gE * ra.mu[3 * j + a] - (g_efield ? g_efield[3 * j + a] : 0.0);
  for (int t = 0; t < 6; t++) {
    const double w = (t == 0 || t == 3 || t == 5) ? 2.0 : 1.0;
    s.t[t] = gE * ra.theta[6 * j + t] - (g_efgrad ? w * g_efgrad[6 * j + t] : 0.0);
  }
  return s;
}

// Energy of the site's moments in the field of a unit charge at -r (r from
// the charge to the site) and its gradient with respect to r:
//   en = Q f1 - (mu.r) f3 + 3/2 (r.theta.r) f5 - 1/2 tr(theta) f3
//   g  = d en / d r = s1 r - f3 mu + 3 f5 theta.r,
//   s1 = -Q f3 + 3 (mu.r) f5 + 3/2 tr(theta) f5 - 15/2 (r.theta.r) f7
DEV void pair_energy_grad(const Site& s, double x, double y, double z, const RadialK& R, double& en, double g[3]) {
  const double md = s.m[0] * x + s.m[1] * y + s.m[2] * z;
  const double thx = s.t[0] * x + s.t[1] * y + s.t[2] * z;
  const double thy = s.t[1] * x + s.t[3] * y + s.t[4] * z;
  const double thz = s.t[2] * x + s.t[4] * y + s.t[5] * z;
  const double dtd = x * thx + y * thy + z * thz;
  const double tr = s.t[0] + s.t[3] + s.t[5];
  en = s.Q * R.f1 - md * R.f3 + 1.5 * dtd * R.f5 - 0.5 * tr * R.f3;
  const double s1 = -s.Q * R.f3 + 3.0 * md * R.f5 + 1.5 * tr * R.f5 - 7.5 * dtd * R.f7;
  const double s3 = 3.0 * R.f5;
  g[0] = s1 * x - R.f3 * s.m[0] + s3 * thx;
  g[1] = s1 * y - R.f3 * s.m[1] + s3 * thy;
  g[2] = s1 * z - R.f3 * s.m[2] + s3 * thz;
}

// potential, gradient and half Hessian at the site of a charge qs at -r
DEV void pair_field(double qs, double x, double y, double z, const RadialK& R, double* F) {
  F[0] += qs * R.f1;
  F[1] -= qs * x * R.f3;
  F[2] -= qs * y * R.f3;
  F[3] -= qs * z * R.f3;
  const double h5 = 1.5 * qs * R.f5, h3 = 0.5 * qs * R.f3;
  F[4] += h5 * x * x - h3;
  F[5] += h5 * x * y;
  F[6] += h5 * x * z;
  F[7] += h5 * y * y - h3;
  F[8] += h5 * y * z;
  F[9] += h5 * z * z - h3;
}

template <int N>
DEV void region_block_sum(double (&v)[N], double (&out)[N]) {
  __shared__ double red[4][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < N; t++) {
    double s = v[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) red[wave][t] = s;
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < N; t++) out[t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
  __syncthreads();
}

// Geometric centre of the QM atoms (every block computes the same value in
// the same order).  Called by all 256 threads.
DEV void qm_centre(int nq, const double* __restrict__ qm_xyz, double (&C)[3]) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < nq; j += 256)
    for (int a = 0; a < 3; a++) v[a] += qm_xyz[3 * j + a];
  region_block_sum<3>(v, C);
  for (int a = 0; a < 3; a++) C[a] /= (double)nq;
}

// translate n of offset d along one axis
DEV double tr_coord(double d, int n, double L) { return d + (double)n * L; }

DEV bool in_region(const RegionArgs& ra, const double d[3], int nx, int ny, int nz) {
  const double x = tr_coord(d[0], nx, ra.box[0]), y = tr_coord(d[1], ny, ra.box[1]), z = tr_coord(d[2], nz, ra.box[2]);
  return x * x + y * y + z * z < ra.r_region * ra.r_region;
}

// Range of n with |c + n L| < R possible along one axis (at most 2 R / L + 1
// values: the radii are validated against the box on the host).  The bounds
// are checked before the conversion to int: a NaN offset (NaN input) or one
// beyond 2^30 box lengths gives an empty range, so no loop runs away.
DEV void n_range(double c, double R, double L, int& lo, int& hi) {
  const double a = ceil((-R - c) / L), b = floor((R - c) / L);
  if (!(a >= -1073741824.0 && b <= 1073741824.0)) {
    lo = 1;
    hi = 0;
    return;
  }
  lo = (int)a;
  hi = (int)b;
}

// nearest lattice index of x (in box lengths), 0 for NaN or beyond 2^30
DEV int nearest_n(double x) { return fabs(x) <= 1073741824.0 ? (int)rint(x) : 0; }

// ------------------------------------------------------------------ preparation
// Work arrays of one region call (RegionWork):
//   cen = (C, max_j |R_j - C|), C the mean QM position;
//   rd[i] = (d, q_i): MM atom i's offset from C reduced to its nearest
//           translate (|d_a| <= L_a/2, so |d| is the distance of the nearest
//           translate to C), and its charge;
//   rk[i] = kappa_i (0: point charge);
//   rf[i] = bit 0: a translate lies in region I (exactly when |d| < r_region);
//           bit 1: a Gaussian charge that may come within r_gauss of a site
//           (|d| < max_j |R_j - C| + r_gauss).
// One thread per MM atom; every block also forms C and the QM extent (the
// same values in the same order), block 0 stores them for later kernels.
__global__ __launch_bounds__(256) void k_region_prep(RegionArgs ra, RegionWork rw, const double* __restrict__ gE_p,
                                                     const double* __restrict__ g_phi,
                                                     const double* __restrict__ g_efield,
                                                     const double* __restrict__ g_efgrad) {
  double C[3];
  qm_centre(ra.nq, ra.qm_xyz, C);
  if (blockIdx.x == 0) {
    // the sites' offsets from C and their moments (the forward pass passes no
    // upstream gradients: gE = 1 and the moments themselves)
    const double gE = gE_p ? *gE_p : 1.0;
    for (int j = threadIdx.x; j < ra.nq; j += 256) {
      const Site st = eff_site(ra, j, gE, g_phi, g_efield, g_efgrad);
      double* p = rw.site + (size_t)j * kRegionSite;
      for (int a = 0; a < 3; a++) p[a] = ra.qm_xyz[3 * j + a] - C[a];
      p[3] = st.Q;
      for (int a = 0; a < 3; a++) p[4 + a] = st.m[a];
      for (int t = 0; t < 6; t++) p[7 + t] = st.t[t];
    }
  }
  __shared__ double rmax[256];
  double m = 0.0;
  for (int j = threadIdx.x; j < ra.nq; j += 256) {
    const double x = ra.qm_xyz[3 * j] - C[0], y = ra.qm_xyz[3 * j + 1] - C[1], z = ra.qm_xyz[3 * j + 2] - C[2];
    m = fmax(m, sqrt(x * x + y * y + z * z));
  }
  rmax[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + o]);
    __syncthreads();
  }
  const double rq = rmax[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rw.cen[0] = C[0];
    rw.cen[1] = C[1];
    rw.cen[2] = C[2];
    rw.cen[3] = rq;
  }
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ra.nm) return;
  double d[3];
  for (int a = 0; a < 3; a++) {
    const double L = ra.box[a];
    const double v = ra.mm_xyz[3 * i + a] - C[a];
    d[a] = v - L * rint(v / L);
  }
  const double kap = ra.kappa ? fmax(ra.kappa[i], 0.0) : 0.0;
  const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  int f = (d2 < ra.r_region * ra.r_region) ? 1 : 0;
  const double reach = rq + ra.r_gauss;
  if (kap > 0.0 && ra.r_gauss > 0.0 && d2 < reach * reach) f |= 2;
  rw.rd[i] = make_double4(d[0], d[1], d[2], ra.mm_q[i]);
  rw.rk[i] = kap;
  rw.rf[i] = f;
}

// Visit every (translate, kappa) pair of an MM atom (offset d, flags f) with
// the site at offset s (= R_j - C): its region-I translates with kappa = 0,
// and for a Gaussian charge its region-II translates within r_gauss of the
// site.  fn(x, y, z, r2, kappa) receives r = R_j - R_i,n.  A radius of at
// most half the smallest box edge admits only the nearest translate (to C,
// or to the site), which skips the range loops.
template <typename Fn>
DEV void for_each_pair(const RegionArgs& ra, const double d[3], int f, double kap, const double s[3], Fn&& fn) {
  int lo[3], hi[3];
  if (f & 1) {
    if (ra.r_region <= ra.half_min) {
      const double x = s[0] - d[0], y = s[1] - d[1], z = s[2] - d[2];
      const double r2 = x * x + y * y + z * z;
      if (r2 > 0.0) fn(x, y, z, r2, 0.0);
    } else {
      for (int a = 0; a < 3; a++) n_range(d[a], ra.r_region, ra.box[a], lo[a], hi[a]);
      for (int nx = lo[0]; nx <= hi[0]; nx++)
        for (int ny = lo[1]; ny <= hi[1]; ny++)
          for (int nz = lo[2]; nz <= hi[2]; nz++) {
            if (!in_region(ra, d, nx, ny, nz)) continue;
            const double x = s[0] - tr_coord(d[0], nx, ra.box[0]);
            const double y = s[1] - tr_coord(d[1], ny, ra.box[1]);
            const double z = s[2] - tr_coord(d[2], nz, ra.box[2]);
            const double r2 = x * x + y * y + z * z;
            if (r2 > 0.0) fn(x, y, z, r2, 0.0);
          }
    }
  }
  if (!(f & 2)) return;
  const double RG = ra.r_gauss;
  // r = s - (d + n L): |s_a - d_a - n L_a| < RG
  if (RG <= ra.half_min) {
    int n[3];
    for (int a = 0; a < 3; a++) n[a] = nearest_n((s[a] - d[a]) * ra.inv_box[a]);
    const double x = s[0] - tr_coord(d[0], n[0], ra.box[0]);
    const double y = s[1] - tr_coord(d[1], n[1], ra.box[1]);
    const double z = s[2] - tr_coord(d[2], n[2], ra.box[2]);
    const double r2 = x * x + y * y + z * z;
    if (r2 < RG * RG && r2 > 0.0 && !in_region(ra, d, n[0], n[1], n[2])) fn(x, y, z, r2, kap);
    return;
  }
  for (int a = 0; a < 3; a++) n_range(d[a] - s[a], RG, ra.box[a], lo[a], hi[a]);
  for (int nx = lo[0]; nx <= hi[0]; nx++)
    for (int ny = lo[1]; ny <= hi[1]; ny++)
      for (int nz = lo[2]; nz <= hi[2]; nz++) {
        const double x = s[0] - tr_coord(d[0], nx, ra.box[0]);
        const double y = s[1] - tr_coord(d[1], ny, ra.box[1]);
        const double z = s[2] - tr_coord(d[2], nz, ra.box[2]);
        const double r2 = x * x + y * y + z * z;
        if (!(r2 < RG * RG) || !(r2 > 0.0) || in_region(ra, d, nx, ny, nz)) continue;
        fn(x, y, z, r2, kap);
      }
}

// site j as the pair kernels use it: offset from C and (effective) moments
DEV Site load_site(const RegionWork& rw, int j, double (&s)[3]) {
  const double* p = rw.site + (size_t)j * kRegionSite;
  Site st;
  for (int a = 0; a < 3; a++) s[a] = p[a];
  st.Q = p[3];
  for (int a = 0; a < 3; a++) st.m[a] = p[4 + a];
  for (int t = 0; t < 6; t++) st.t[t] = p[7 + t];
  return st;
}

// ------------------------------------------------------------------ QM side
// Grid (QM site, MM chunk).  Each block sums, over the flagged MM atoms of
// its chunk, the potential, gradient and half Hessian of the subtracted
// charges at the site (10 values) and, with BWD = 1, the site's position
// gradient with the effective moments (3 more); partial sums per chunk go to
// rw.part[site][chunk][13].
template <int BWD>
__global__ __launch_bounds__(256) void k_region_qm(RegionArgs ra, RegionWork rw, int chunk) {
  const int j = blockIdx.x;
  double s[3];
  const Site st = load_site(rw, j, s);
  constexpr int NV = BWD ? 13 : 10;
  double acc[NV];
#pragma unroll
  for (int t = 0; t < NV; t++) acc[t] = 0.0;
  const int i0 = blockIdx.y * chunk, i1 = min(ra.nm, i0 + chunk);
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const int f = rw.rf[i];
    if (!f) continue;
    const double4 dq = rw.rd[i];
    const double d[3] = {dq.x, dq.y, dq.z};
    const double qs = -dq.w;  // subtracted
    for_each_pair(ra, d, f, rw.rk[i], s, [&](double x, double y, double z, double r2, double k) {
      const RadialK R = radial_k(r2, k);
      pair_field(qs, x, y, z, R, acc);
      if (BWD) {
        double en, g[3];
        pair_energy_grad(st, x, y, z, R, en, g);
        acc[10] += qs * g[0];
        acc[11] += qs * g[1];
        acc[12] += qs * g[2];
      }
    });
  }
  double tot[NV];
  region_block_sum<NV>(acc, tot);
  if (threadIdx.x == 0) {
    double* o = rw.part + ((size_t)j * gridDim.y + blockIdx.y) * kRegionNV;
    for (int t = 0; t < NV; t++) o[t] = tot[t];
  }
}

// ------------------------------------------------------------------ MM side (adjoint)
// dL/dR_i and dL/dq_i of the subtracted pairs with the effective moments.
// The flagged atoms of a wave are taken one after another; for each, the 64
// lanes share its QM sites and a butterfly sum (fixed order) combines them.
__global__ __launch_bounds__(256) void k_region_mm(RegionArgs ra, RegionWork rw, double* __restrict__ g_mm_xyz,
                                                   double* __restrict__ g_mm_q) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int f = (i < ra.nm) ? rw.rf[i] : 0;
  unsigned long long mask = __ballot(f != 0);
  while (mask) {
    const int src = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    const int ii = i - lane + src;
    const double4 dq = rw.rd[ii];
    const double d[3] = {dq.x, dq.y, dq.z};
    const double q = dq.w, kap = rw.rk[ii];
    const int ff = rw.rf[ii];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = lane; j < ra.nq; j += 64) {
      double s[3];
      const Site st = load_site(rw, j, s);
      for_each_pair(ra, d, ff, kap, s, [&](double x, double y, double z, double r2, double k) {
        const RadialK R = radial_k(r2, k);
        double en, g[3];
        pair_energy_grad(st, x, y, z, R, en, g);
        // pair term of L: -q en(r), r = R_j - R_i: d/dR_i = +q g, d/dq = -en
        v[0] += q * g[0];
        v[1] += q * g[1];
        v[2] += q * g[2];
        v[3] -= en;
      });
    }
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v[t] += __shfl_xor(v[t], o, 64);
    if (lane == src) {
      g_mm_xyz[3 * ii] += v[0];
      g_mm_xyz[3 * ii + 1] += v[1];
      g_mm_xyz[3 * ii + 2] += v[2];
      if (g_mm_q) g_mm_q[ii] += v[3];
    }
  }
}

// ------------------------------------------------------------------ unit-cell QM-QM pairs and site outputs
// Bare tensors up to order 3 of 1/|r|, r = R_a - R_b:
//   p0 = 1/r, p1 = -r/r^3, p2 = 1/2 (3 r r / r^5 - I / r^3),
//   p3_abc = 1/2 [ (d_ab r_c + d_ac r_b + d_bc r_a) / r^5 - 5 r_a r_b r_c / r^7 ]
// The pair form (both orientations of each pair, order-2 truncated):
//   P = Qa Qb p0 + (Qb mu_a - Qa mu_b).p1 + (Qb th_a + Qa th_b):p2 - 2 mu_a.p2.mu_b
// Site a collects -1/2 P(a, b) for the energy and -dP(a, b)/d(its own inputs)
// over b != a (P(a,b) = P(b,a), so the ordered-pair half cancels).
// v[0] energy, v[1..3] position, v[4] Q, v[5..7] mu, v[8..13] stored theta.
static constexpr int kQQ = 14;

DEV void qq_pair(const RegionArgs& ra, int a, int b, bool bwd, double (&v)[kQQ]) {
  double r[3];
  for (int c = 0; c < 3; c++) r[c] = ra.qm_xyz[3 * a + c] - ra.qm_xyz[3 * b + c];
  const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  if (!(r2 > 0.0)) return;
  const RadialK R = radial_k(r2, 0.0);
  const double Qa = ra.Q[a], Qb = ra.Q[b];
  double ma[3], mb[3], ta[3][3], tb[3][3];
  for (int c = 0; c < 3; c++) {
    ma[c] = ra.mu[3 * a + c];
    mb[c] = ra.mu[3 * b + c];
  }
  {
    const double* t = ra.theta + 6 * a;
    ta[0][0] = t[0]; ta[0][1] = ta[1][0] = t[1]; ta[0][2] = ta[2][0] = t[2];
    ta[1][1] = t[3]; ta[1][2] = ta[2][1] = t[4]; ta[2][2] = t[5];
    t = ra.theta + 6 * b;
    tb[0][0] = t[0]; tb[0][1] = tb[1][0] = t[1]; tb[0][2] = tb[2][0] = t[2];
    tb[1][1] = t[3]; tb[1][2] = tb[2][1] = t[4]; tb[2][2] = t[5];
  }
  double p1[3], p2[3][3];
  for (int c = 0; c < 3; c++) p1[c] = -r[c] * R.f3;
  for (int c = 0; c < 3; c++)
    for (int d = 0; d < 3; d++) p2[c][d] = 0.5 * (3.0 * r[c] * r[d] * R.f5 - (c == d ? R.f3 : 0.0));
  const double p0 = R.f1;
  double P = Qa * Qb * p0;
  double w[3][3];  // Qb th_a + Qa th_b
  for (int c = 0; c < 3; c++) P += (Qb * ma[c] - Qa * mb[c]) * p1[c];
  for (int c = 0; c < 3; c++)
    for (int d = 0; d < 3; d++) {
      w[c][d] = Qb * ta[c][d] + Qa * tb[c][d];
      P += w[c][d] * p2[c][d] - 2.0 * ma[c] * p2[c][d] * mb[d];
    }
  v[0] -= 0.5 * P;
  if (!bwd) return;
  // dP/dr_g: order-3 tensor contracted on the fly
  for (int g = 0; g < 3; g++) {
    double dg = Qa * Qb * p1[g];
    for (int c = 0; c < 3; c++) dg += (Qb * ma[c] - Qa * mb[c]) * 2.0 * p2[c][g];
    for (int c = 0; c < 3; c++)
      for (int d = 0; d < 3; d++) {
        double sm = 0.0;
        if (c == d) sm += r[g];
        if (c == g) sm += r[d];
        if (d == g) sm += r[c];
        const double p3 = 0.5 * (sm * R.f5 - 5.0 * r[c] * r[d] * r[g] * R.f7);
        dg += (w[c][d] - 2.0 * ma[c] * mb[d]) * 3.0 * p3;
      }
    v[1 + g] -= dg;
  }
  double dQ = Qb * p0;
  for (int c = 0; c < 3; c++) dQ -= mb[c] * p1[c];
  for (int c = 0; c < 3; c++)
    for (int d = 0; d < 3; d++) dQ += tb[c][d] * p2[c][d];
  v[4] -= dQ;
  for (int c = 0; c < 3; c++) {
    double dm = Qb * p1[c];
    for (int d = 0; d < 3; d++) dm -= 2.0 * p2[c][d] * mb[d];
    v[5 + c] -= dm;
  }
  // stored theta numbers: off-diagonals collect both matrix elements
  v[8] -= Qb * p2[0][0];
  v[9] -= 2.0 * Qb * p2[0][1];
  v[10] -= 2.0 * Qb * p2[0][2];
  v[11] -= Qb * p2[1][1];
  v[12] -= 2.0 * Qb * p2[1][2];
  v[13] -= Qb * p2[2][2];
}

// One wave per site a: the lanes share the QM-QM pairs (a, b) and the sums
// of the chunk partials of the MM terms; lane 0 applies the results.
// BWD = 0: add the MM field to phi, efield, efgrad; e_site[a] = the site's
// MM energy + its QM-QM pair energy.  BWD = 1: add the position gradients and
// gE x (field + QM-QM moment derivatives) = dE/d(moments).
template <int BWD>
__global__ __launch_bounds__(64) void k_region_site(RegionArgs ra, RegionWork rw, int nchunk,
                                                    const double* __restrict__ gE_p, double* __restrict__ e_site,
                                                    double* __restrict__ phi, double* __restrict__ efield,
                                                    double* __restrict__ efgrad, double* __restrict__ g_qm_xyz,
                                                    double* __restrict__ g_Q, double* __restrict__ g_mu,
                                                    double* __restrict__ g_theta) {
  const int a = blockIdx.x, lane = threadIdx.x;
  double v[kQQ];
#pragma unroll
  for (int t = 0; t < kQQ; t++) v[t] = 0.0;
  for (int b = lane; b < ra.nq; b += 64)
    if (b != a) qq_pair(ra, a, b, BWD != 0, v);
#pragma unroll
  for (int t = 0; t < kQQ; t++)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[t] += __shfl_xor(v[t], o, 64);
  // lane t < 13 sums partial t over the chunks
  constexpr int NV = BWD ? 13 : 10;
  double mine = 0.0;
  if (lane < NV)
    for (int c = 0; c < nchunk; c++) mine += rw.part[((size_t)a * nchunk + c) * kRegionNV + lane];
  double tot[NV];
#pragma unroll
  for (int t = 0; t < NV; t++) tot[t] = __shfl(mine, t, 64);
  if (lane != 0) return;
  if (!BWD) {
    if (phi) phi[a] += tot[0];
    if (efield)
      for (int c = 0; c < 3; c++) efield[3 * a + c] -= tot[1 + c];
    if (efgrad)
      for (int t = 0; t < 6; t++) efgrad[6 * a + t] -= 2.0 * tot[4 + t];
    double e = ra.Q[a] * tot[0];
    for (int c = 0; c < 3; c++) e += ra.mu[3 * a + c] * tot[1 + c];
    for (int t = 0; t < 6; t++) e += ((t == 0 || t == 3 || t == 5) ? 1.0 : 2.0) * ra.theta[6 * a + t] * tot[4 + t];
    e_site[a] = e + v[0];
  } else {
    const double gE = gE_p ? *gE_p : 1.0;
    for (int c = 0; c < 3; c++) g_qm_xyz[3 * a + c] += tot[10 + c] + gE * v[1 + c];
    g_Q[a] += gE * (tot[0] + v[4]);
    for (int c = 0; c < 3; c++) g_mu[3 * a + c] += gE * (tot[1 + c] + v[5 + c]);
    for (int t = 0; t < 6; t++)
      g_theta[6 * a + t] += gE * (((t == 0 || t == 3 || t == 5) ? 1.0 : 2.0) * tot[4 + t] + v[8 + t]);
  }
}

// energy += sum of the site energies (one block, fixed order)
__global__ __launch_bounds__(256) void k_region_energy(int nq, const double* __restrict__ e_site,
                                                       double* __restrict__ energy) {
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < nq; j += 256) v[0] += e_site[j];
  double tot[1];
  region_block_sum<1>(v, tot);
  if (threadIdx.x == 0) energy[0] += tot[0];
}

static void region_chunks(int nm, int& nchunk, int& chunk) {
  nchunk = std::max(1, std::min(kRegionMaxChunks, (nm + 2047) / 2048));
  chunk = std::max(256, ((nm + nchunk - 1) / nchunk + 255) / 256 * 256);
}

static void launch_region_common(const RegionArgs& ra, const RegionWork& rw, const double* gE, const double* g_phi,
                                 const double* g_efield, const double* g_efgrad, hipStream_t s) {
  hipLaunchKernelGGL(k_region_prep, dim3(std::max(1, (ra.nm + 255) / 256)), dim3(256), 0, s, ra, rw, gE, g_phi,
                     g_efield, g_efgrad);
}

hipError_t launch_region_forward(const RegionArgs& ra, const RegionWork& rw, double* e_site, double* energy,
                                 double* phi, double* efield, double* efgrad, hipStream_t s) {
  if (ra.nq == 0) return hipSuccess;
  int nchunk, chunk;
  region_chunks(ra.nm, nchunk, chunk);
  launch_region_common(ra, rw, nullptr, nullptr, nullptr, nullptr, s);
  hipLaunchKernelGGL((k_region_qm<0>), dim3(ra.nq, nchunk), dim3(256), 0, s, ra, rw, chunk);
  hipLaunchKernelGGL((k_region_site<0>), dim3(ra.nq), dim3(64), 0, s, ra, rw, nchunk, nullptr, e_site, phi, efield,
                     efgrad, nullptr, nullptr, nullptr, nullptr);
  hipLaunchKernelGGL(k_region_energy, dim3(1), dim3(256), 0, s, ra.nq, (const double*)e_site, energy);
  return hipGetLastError();
}

hipError_t launch_region_backward(const RegionArgs& ra, const RegionWork& rw, const double* gE, const double* g_phi,
                                  const double* g_efield, const double* g_efgrad, double* g_qm_xyz, double* g_Q,
                                  double* g_mu, double* g_theta, double* g_mm_xyz, double* g_mm_q, hipStream_t s) {
  if (ra.nq == 0) return hipSuccess;
  int nchunk, chunk;
  region_chunks(ra.nm, nchunk, chunk);
  launch_region_common(ra, rw, gE, g_phi, g_efield, g_efgrad, s);
  hipLaunchKernelGGL((k_region_qm<1>), dim3(ra.nq, nchunk), dim3(256), 0, s, ra, rw, chunk);
  hipLaunchKernelGGL((k_region_site<1>), dim3(ra.nq), dim3(64), 0, s, ra, rw, nchunk, gE, nullptr, nullptr, nullptr,
                     nullptr, g_qm_xyz, g_Q, g_mu, g_theta);
  if (ra.nm > 0)
    hipLaunchKernelGGL(k_region_mm, dim3((ra.nm + 255) / 256), dim3(256), 0, s, ra, rw, g_mm_xyz, g_mm_q);
  return hipGetLastError();
}

__global__ void k_zero_part(double* __restrict__ p, int n) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0.0;
}

// ------------------------------------------------------------------ charge-octupole error estimate
// Err(R_k) = sum over MM translates with R_k <= |R_i,n - C| < r_outer of
// q_i sum_j Omega_j : T_abc(R_j - R_i,n), for R_k = r_first + k r_step
// (main text, Error Control; SI, T_abc = 1/3 d T_ab).  With the raw third
// moment Omega (symmetric; ten stored components) and its trace vector
// t_a = sum_b Omega_abb:
//   Omega : T(r) = -[5 Omega(r,r,r) - 3 r^2 (t.r)] / (2 r^7).
// Grid (MM blocks, candidate chunks of kOctBins): each thread takes one MM
// atom, visits its translates inside r_outer with the QM sites staged in LDS,
// and adds each translate's term to the candidates it lies beyond; per-block
// partial sums go to part[k][block], reduced in a fixed order afterwards.
static constexpr int kOctBins = 16;

DEV double octupole_energy(const double* om, double x, double y, double z) {
  const double r2 = x * x + y * y + z * z;
  const double rrr = om[0] * x * x * x + 3.0 * om[1] * x * x * y + 3.0 * om[2] * x * x * z + 3.0 * om[3] * x * y * y +
                     6.0 * om[4] * x * y * z + 3.0 * om[5] * x * z * z + om[6] * y * y * y + 3.0 * om[7] * y * y * z +
                     3.0 * om[8] * y * z * z + om[9] * z * z * z;
  const double tr = (om[0] + om[3] + om[5]) * x + (om[1] + om[6] + om[8]) * y + (om[2] + om[7] + om[9]) * z;
  const double r7 = r2 * r2 * r2 * sqrt(r2);
  return -(5.0 * rrr - 3.0 * r2 * tr) / (2.0 * r7);
}

__global__ __launch_bounds__(256) void k_octupole(OctArgs oa, double* __restrict__ part) {
  __shared__ double sp[256][13];  // site offset from the centre (3), Omega (10)
  double C[3];
  qm_centre(oa.nq, oa.qm_xyz, C);
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < oa.nm;
  const int k0 = blockIdx.y * kOctBins;
  double d[3] = {0.0, 0.0, 0.0};
  double q = 0.0;
  if (valid) {
    for (int a = 0; a < 3; a++) {
      const double L = oa.box[a];
      const double v = oa.mm_xyz[3 * i + a] - C[a];
      d[a] = v - L * rint(v / L);
    }
    q = oa.mm_q[i];
  }
  double acc[kOctBins];
#pragma unroll
  for (int t = 0; t < kOctBins; t++) acc[t] = 0.0;
  const double Ro = oa.r_outer;
  for (int t0 = 0; t0 < oa.nq; t0 += 256) {
    const int jl = t0 + threadIdx.x;
    __syncthreads();
    if (jl < oa.nq) {
      for (int a = 0; a < 3; a++) sp[threadIdx.x][a] = oa.qm_xyz[3 * jl + a] - C[a];
      for (int c = 0; c < 10; c++) sp[threadIdx.x][3 + c] = oa.omega[10 * jl + c];
    }
    __syncthreads();
    if (!valid) continue;
    const int nt = min(256, oa.nq - t0);
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) n_range(d[a], Ro, oa.box[a], lo[a], hi[a]);
    for (int nx = lo[0]; nx <= hi[0]; nx++)
      for (int ny = lo[1]; ny <= hi[1]; ny++)
        for (int nz = lo[2]; nz <= hi[2]; nz++) {
          const double tx = tr_coord(d[0], nx, oa.box[0]), ty = tr_coord(d[1], ny, oa.box[1]),
                       tz = tr_coord(d[2], nz, oa.box[2]);
          const double D2 = tx * tx + ty * ty + tz * tz;
          if (!(D2 < Ro * Ro)) continue;
          const double D = sqrt(D2);
          double e = 0.0;
          for (int jj = 0; jj < nt; jj++) {
            const double x = sp[jj][0] - tx, y = sp[jj][1] - ty, z = sp[jj][2] - tz;
            if (x * x + y * y + z * z > 0.0) e += octupole_energy(&sp[jj][3], x, y, z);
          }
          e *= q;
#pragma unroll
          for (int kk = 0; kk < kOctBins; kk++) {
            const int k = k0 + kk;
            if (k < oa.n_r && D >= oa.r_first + (double)k * oa.r_step) acc[kk] += e;
          }
        }
  }
  double tot[kOctBins];
  region_block_sum<kOctBins>(acc, tot);
  if (threadIdx.x == 0)
    for (int kk = 0; kk < kOctBins; kk++)
      if (k0 + kk < oa.n_r) part[(size_t)(k0 + kk) * gridDim.x + blockIdx.x] = tot[kk];
}

// err[k] = sum of the block partials in a fixed order: tpk threads per
// candidate each sum every tpk-th block, then one of them adds the tpk sums;
// r_cut = the first R_k whose estimate and the next one's are below eps in
// magnitude, -1 if none.
__global__ __launch_bounds__(256) void k_octupole_final(OctArgs oa, int nblocks, const double* __restrict__ part,
                                                        double eps, double* __restrict__ err,
                                                        double* __restrict__ r_cut) {
  __shared__ double sub[256];
  __shared__ double se[kMaxOctCandidates];
  int np2 = 1;
  while (np2 < oa.n_r) np2 <<= 1;
  const int tpk = 256 / np2;  // n_r <= 256
  const int k = threadIdx.x / tpk, u = threadIdx.x % tpk;
  double s = 0.0;
  if (k < oa.n_r)
    for (int b = u; b < nblocks; b += tpk) s += part[(size_t)k * nblocks + b];
  sub[threadIdx.x] = s;
  __syncthreads();
  if (k < oa.n_r && u == 0) {
    double t = 0.0;
    for (int v = 0; v < tpk; v++) t += sub[threadIdx.x + v];
    se[k] = t;
    err[k] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0 || !r_cut) return;
  double pick = -1.0;
  for (int kk = 0; kk + 1 < oa.n_r; kk++)
    if (fabs(se[kk]) < eps && fabs(se[kk + 1]) < eps) {
      pick = oa.r_first + (double)kk * oa.r_step;
      break;
    }
  r_cut[0] = pick;
}

hipError_t launch_octupole(const OctArgs& oa, double* part, double eps, double* err, double* r_cut, hipStream_t s) {
  const int nb = oa.nm > 0 ? (oa.nm + 255) / 256 : 0;
  if (nb > 0 && oa.nq > 0) {
    hipLaunchKernelGGL(k_octupole, dim3(nb, (oa.n_r + kOctBins - 1) / kOctBins), dim3(256), 0, s, oa, part);
  } else {
    // no pairs: every estimate is zero
    hipLaunchKernelGGL(k_zero_part, dim3(1), dim3(256), 0, s, part, oa.n_r);
  }
  hipLaunchKernelGGL(k_octupole_final, dim3(1), dim3(256), 0, s, oa, (nb > 0 && oa.nq > 0) ? nb : 1,
                     (const double*)part, eps, err, r_cut);
  return hipGetLastError();
}

}  // namespace mpe
