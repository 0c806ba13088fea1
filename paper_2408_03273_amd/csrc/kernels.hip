// HIP kernels for gfx950 of the multipolar Ewald QM/MM coupling.
//
// Paper: Methods (periodic QM/MM multipole energy, Fock potential and
// nuclear gradient) and Supporting Information "Multipolar Ewald"
// (screened tensors with f1..f7, reciprocal-space tensors, self terms).
//
// Reciprocal vectors are stored per frame on the box [0,mx] x [-my,my] x
// [-mz,mz]; only the half space nx>0 | (nx=0 & ny>0) | (nx=ny=0 & nz>0)
// carries weight (2 x (4 pi/V) e^{-k^2/4a^2}/k^2); the rest is masked.
// Flat index k = col*NZ + (nz+mz), col = nx*NY + (ny+my).
#include <math.h>

#include <algorithm>
#include <initializer_list>
#include <type_traits>

#include "ewald_internal.h"

namespace mpe {

#define DEV __device__ __forceinline__

static constexpr double kPi = 3.14159265358979323846;

DEV int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

DEV double uniform_double(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffu));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The descriptor is selected between a kernel argument and device memory, so
// the compiler cannot see that it is wave-uniform; say so explicitly, which
// keeps the per-atom table reads of the hot loops on the scalar unit.
DEV FrameDev get_frame(const FrameArg& fa, int f) {
  FrameDev r = fa.frames ? fa.frames[f] : fa.f0;
  for (int a = 0; a < 3; a++) {
    r.box[a] = uniform_double(r.box[a]);
    r.inv_box[a] = uniform_double(r.inv_box[a]);
  }
  r.nq = uniform_int(r.nq);
  r.nm = uniform_int(r.nm);
  r.qoff = uniform_int(r.qoff);
  r.moff = uniform_int(r.moff);
  r.slot_base = uniform_int(r.slot_base);
  for (int a = 0; a < 3; a++) r.nc[a] = uniform_int(r.nc[a]);
  r.cell_base = uniform_int(r.cell_base);
  r.orig = uniform_int(r.orig);
  r.nimg = uniform_int(r.nimg);
  return r;
}

DEV double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

DEV double wrap_coord(double x, double L) {
  double w = x - L * floor(x / L);
  if (w >= L) w -= L;
  if (w < 0.0) w += L;
  return w;
}

DEV bool in_half_space(int nx, int ny, int nz) { return nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0))); }

// ------------------------------------------------------------------ reductions
DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum N values over a 256-thread block through red (4 N doubles of LDS);
// thread 0 gets the totals in out[].
template <int N>
DEV void block_sum256_lds(double (&v)[N], double (&out)[N], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < N; t++) {
    double s = wave_sum(v[t]);
    if (lane == 0) red[wave * N + t] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < N; t++) out[t] = red[t] + red[N + t] + red[2 * N + t] + red[3 * N + t];
  }
  __syncthreads();
}

template <int N>
DEV void block_sum256(double (&v)[N], double (&out)[N]) {
  __shared__ double red[4 * N];
  block_sum256_lds<N>(v, out, red);
}

// ------------------------------------------------------------------ zero fill
__global__ void k_zero(double* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

hipError_t launch_zero(double* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fixed-order sums (deterministic mode)
// dst[row * dst_stride + map.off[t]] += sum over b of src[...] in the order of b:
//   mode 0: row = frame f, src[(f * nb + b) * stride + t], b < nb;
//   mode 1: row = packed QM row r = qoff + j of each site j of each frame,
//           src[(r * nb + b) * stride + t], b < nb;
//   mode 2: row = frame f, src[(qoff + b) * stride + t], b < nq (the frame's QM rows).
__global__ __launch_bounds__(64) void k_det_reduce(FrameArg fa, int mode, const double* __restrict__ src, int nb,
                                                   int stride, DetMap map, double* __restrict__ dst,
                                                   int dst_stride) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int t = threadIdx.x;
  if (t >= map.n) return;
  size_t row, base;
  int count = nb, step = stride;
  if (mode == 1) {
    const int j = blockIdx.x;
    if (j >= fr.nq) return;
    row = (size_t)(fr.qoff + j);
    base = row * nb * stride;
  } else if (mode == 2) {
    row = (size_t)f;
    base = (size_t)fr.qoff * stride;
    count = fr.nq;
  } else {
    row = (size_t)f;
    base = (size_t)f * nb * stride;
  }
  double sum = 0.0;
  for (int b = 0; b < count; b++) sum += src[base + (size_t)b * step + t];
  dst[row * dst_stride + map.off[t]] += sum;
}

hipError_t launch_det_reduce(const FrameArg& fa, int mode, int rows, const double* src, int nb, int stride,
                             const DetMap& map, double* dst, int dst_stride, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_det_reduce, dim3(mode == 1 ? rows : 1, fa.n_frames), dim3(64), 0, s, fa, mode, src, nb,
                     stride, map, dst, dst_stride);
  return hipGetLastError();
}

static DetMap det_map(std::initializer_list<int> offs) {
  DetMap m{};
  m.n = 0;
  for (int o : offs) m.off[m.n++] = o;
  return m;
}

static DetMap det_range(DetMap m, int first, int count) {
  for (int t = 0; t < count; t++) m.off[m.n++] = first + t;
  return m;
}

// ------------------------------------------------------------------ preparation
// Wrap positions into the cell, store them SoA with the charges, and sum the
// charges of each subsystem of the frame.
__global__ __launch_bounds__(256) void k_prep_pos(FrameArg fa, const double* __restrict__ qm_xyz,
                                                  const double* __restrict__ Q, const double* __restrict__ mm_xyz,
                                                  const double* __restrict__ mm_q, const double* __restrict__ mu,
                                                  const double* __restrict__ theta, double* __restrict__ qm4,
                                                  int cap_qm, double* __restrict__ mm4, int cap_mm,
                                                  double* __restrict__ qacc, double* __restrict__ qeff, int unit_eff,
                                                  double* __restrict__ facc, double* __restrict__ rpart,
                                                  double* __restrict__ det) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int i = blockIdx.x * 256 + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < fr.nm) {
    const int r = fr.moff + i;
    for (int a = 0; a < 3; a++) mm4[(size_t)a * cap_mm + r] = wrap_coord(mm_xyz[3 * (size_t)r + a], fr.box[a]);
    mm4[(size_t)3 * cap_mm + r] = mm_q[r];
    v[0] = mm_q[r];
    // real-space MM adjoint data accumulate with atomics from zero
    if (rpart)
      for (int t = 0; t < 4; t++) rpart[(size_t)r * 4 + t] = 0.0;
  }
  if (i < fr.nq) {
    const int r = fr.qoff + i;
    for (int a = 0; a < 3; a++) qm4[(size_t)a * cap_qm + r] = wrap_coord(qm_xyz[3 * (size_t)r + a], fr.box[a]);
    qm4[(size_t)3 * cap_qm + r] = Q[r];
    v[1] = Q[r];
    // the QM accumulators of this row start from zero
    for (int t = 0; t < QA_STRIDE; t++) qacc[(size_t)r * QA_STRIDE + t] = 0.0;
    if (unit_eff) {
      // effective moments for an upstream gradient of 1 on E only: the moments themselves
      double* o = qeff + 10 * (size_t)r;
      o[0] = Q[r];
      for (int t = 0; t < 3; t++) o[1 + t] = mu[3 * (size_t)r + t];
      for (int t = 0; t < 6; t++) o[4 + t] = theta[6 * (size_t)r + t];
    }
  }
  double tot[2];
  block_sum256<2>(v, tot);
  if (threadIdx.x == 0) {
    if (det) {
      // every block writes its partial sums (zero past the frame's atoms)
      double* o = det + ((size_t)f * gridDim.x + blockIdx.x) * 3;
      o[0] = tot[0];
      o[1] = tot[1];
      o[2] = unit_eff ? tot[1] : 0.0;
    } else if (blockIdx.x * 256 < max(fr.nm, fr.nq)) {
      atomicAdd(&facc[f * FA_COUNT + FA_QTOT_MM], tot[0]);
      atomicAdd(&facc[f * FA_COUNT + FA_QTOT_QM], tot[1]);
      if (unit_eff) atomicAdd(&facc[f * FA_COUNT + FA_QTOT_EFF], tot[1]);
    }
  }
}

// Per-atom phase tables.  Row layout (complex):
// [e^{i 2pi n x/Lx}, n = 0..mx][e^{i 2pi n y/Ly}, n = -my..my][e^{i 2pi n z/Lz}, n = -mz..mz, then zeros]
// and, for the MM atoms, a real z row [cos(2pi p z/Lz), p = 1..mz][sin(2pi p z/Lz), p = 1..mz]
// (the padding after it is zeroed once at set-up).
// A block builds the rows of kTabAtoms consecutive atoms in LDS: first
// u = e^{i 2pi x/L} per atom and axis (one sincospi each), then one thread
// per run of kTabRun entries of one axis, whose first entry is u^n by binary
// powering (conjugated for n < 0) and the rest by multiplying with u (about
// 2 log2(n) + kTabRun rounding steps in all, ~1e-15 relative); the rows,
// contiguous in memory, are then written out with consecutive threads on
// consecutive entries.
// (run length and LDS row strides chosen so that the 16-byte LDS writes of a
// wave spread over the banks)
static constexpr int kTabRun = 7;
static constexpr int kTabAtoms = 16;
static constexpr int kTabMaxR = 192;    // complex entries per row held in LDS
static constexpr int kTabMaxZ = 64;     // real z entries per row held in LDS
static constexpr int kTabBlocks = 4096;  // blocks of a table pass (several frames share them)

__global__ __launch_bounds__(256) void k_prep_tab(Grid g, FrameArg fa, int qm_side, int with_ez,
                                                  const double* __restrict__ pos4, int cap, double2* __restrict__ tab,
                                                  double* __restrict__ ztab, double2* __restrict__ xy) {
  // complex rows in dynamic LDS, sized for the entries actually built (row
  // stride nc + 1), so that more blocks fit a CU when the z part is not built
  extern __shared__ double2 rowbuf[];
  __shared__ double zrows[kTabAtoms][kTabMaxZ + 1];
  __shared__ double2 base[kTabAtoms][3];
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int n_atoms = qm_side ? fr.nq : fr.nm;
  const int off = qm_side ? fr.qoff : fr.moff;
  const int nc = g.NX + g.NY + (with_ez ? g.NZP : 0);  // complex entries built per row
  const int rs = nc + 1;
  auto rows = [&](int a, int c) -> double2& { return rowbuf[a * rs + c]; };
  const int rx = (g.NX + kTabRun - 1) / kTabRun, ry = (g.NY + kTabRun - 1) / kTabRun,
            rz = with_ez ? (g.NZP + kTabRun - 1) / kTabRun : 0, rr = ztab ? (g.mz + kTabRun - 1) / kTabRun : 0;
  const int runs = rx + ry + rz + rr;
  // The block takes groups of kTabAtoms atoms in turn: the stores of one
  // group drain while the next is built (the barrier after a group's u per
  // atom and axis also orders the previous group's reads of the LDS rows
  // before the new rows are written).
  for (int a0 = blockIdx.x * kTabAtoms; a0 < n_atoms; a0 += gridDim.x * kTabAtoms) {  // uniform over the block
    const int na = min(kTabAtoms, n_atoms - a0);
    if (threadIdx.x < na * 3) {
      const int a = threadIdx.x / 3, ax = threadIdx.x - 3 * a;
      const double x = pos4[(size_t)ax * cap + off + a0 + a] / fr.box[ax];
      double sn, cs;
      sincospi(2.0 * x, &sn, &cs);
      base[a][ax] = make_double2(cs, sn);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < na * runs; t += 256) {
      const int a = t / runs, u = t - a * runs;
      int axis, first, count, n0, limit;
      if (u < rx) {
        axis = 0;
        first = u * kTabRun;
        count = min(kTabRun, g.NX - first);
        n0 = first;
        limit = count;
      } else if (u < rx + ry) {
        axis = 1;
        first = (u - rx) * kTabRun;
        count = min(kTabRun, g.NY - first);
        n0 = first - g.my;
        first += g.NX;
        limit = count;
      } else if (u < rx + ry + rz) {
        axis = 2;
        first = (u - rx - ry) * kTabRun;
        count = min(kTabRun, g.NZP - first);
        n0 = first - g.mz;
        limit = g.NZ - first;  // z entries past NZ are padding
        first += g.NX + g.NY;
      } else {
        axis = 3;  // real z row, p = first+1 ..
        first = (u - rx - ry - rz) * kTabRun;
        count = min(kTabRun, g.mz - first);
        n0 = first + 1;
        limit = count;
      }
      const int ax = axis == 3 ? 2 : axis;
      const double2 step = base[a][ax];
      // v = step^n0
      double2 v = make_double2(1.0, 0.0), pw = step;
      for (int m = n0 < 0 ? -n0 : n0; m; m >>= 1) {
        if (m & 1) v = cmul(v, pw);
        pw = cmul(pw, pw);
      }
      if (n0 < 0) v = cconj(v);
      for (int e = 0; e < count; e++) {
        if (axis == 3) {
          zrows[a][first + e] = v.x;
          zrows[a][g.mz + first + e] = v.y;
        } else {
          rows(a, first + e) = e < limit ? v : make_double2(0.0, 0.0);
        }
        v = cmul(v, step);
      }
    }
    __syncthreads();
    if (with_ez) {
      // whole rows: one contiguous run of na * R entries
      double2* __restrict__ o = tab + (size_t)(off + a0) * g.R;
      for (int e = threadIdx.x; e < na * g.R; e += 256) {
        const int a = e / g.R, c = e - a * g.R;
        o[e] = rows(a, c);
      }
    }
    if (xy) {
      // compact x/y rows (stride NX + NY): one contiguous run of na * NXY entries
      double2* __restrict__ o = xy + (size_t)(off + a0) * g.NXY;
      for (int e = threadIdx.x; e < na * g.NXY; e += 256) {
        const int a = e / g.NXY, c = e - a * g.NXY;
        o[e] = rows(a, c);
      }
    }
    if (ztab) {
      const int zw = 2 * g.mz;
      for (int e = threadIdx.x; e < na * zw; e += 256) {
        const int a = e / zw, c = e - a * zw;
        ztab[(size_t)(off + a0 + a) * g.ZKP + c] = zrows[a][c];
      }
    }
  }
}

// Grids whose rows do not fit the LDS tile: one thread per entry, each from its own sincospi.
__global__ __launch_bounds__(256) void k_prep_tab_direct(Grid g, FrameArg fa, int qm_side, int with_ez,
                                                         const double* __restrict__ pos4, int cap,
                                                         double2* __restrict__ tab, double* __restrict__ ztab,
                                                         double2* __restrict__ xy) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int n_atoms = qm_side ? fr.nq : fr.nm;
  const int off = qm_side ? fr.qoff : fr.moff;
  const int nc = g.NX + g.NY + (with_ez ? g.NZP : 0);
  const int per = nc + (ztab ? g.mz : 0);
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)n_atoms * per) return;
  const int a = (int)(e / per), u = (int)(e - (long)a * per);
  const int row = off + a;
  int ax, n;
  if (u < g.NX) {
    ax = 0;
    n = u;
  } else if (u < g.NX + g.NY) {
    ax = 1;
    n = u - g.NX - g.my;
  } else if (u < nc) {
    ax = 2;
    const int iz = u - g.NX - g.NY;
    if (iz >= g.NZ) {
      tab[(size_t)row * g.R + u] = make_double2(0.0, 0.0);
      return;
    }
    n = iz - g.mz;
  } else {
    ax = 3;
    n = u - nc + 1;
  }
  const int axc = ax == 3 ? 2 : ax;
  const double x = pos4[(size_t)axc * cap + row] / fr.box[axc];
  double sn, cs;
  sincospi(2.0 * (double)n * x, &sn, &cs);
  if (ax == 3) {
    ztab[(size_t)row * g.ZKP + n - 1] = cs;
    ztab[(size_t)row * g.ZKP + g.mz + n - 1] = sn;
  } else {
    if (with_ez || ax == 2) tab[(size_t)row * g.R + u] = make_double2(cs, sn);
    if (xy && ax < 2) xy[(size_t)row * g.NXY + u] = make_double2(cs, sn);
  }
}

// with_ez: full complex rows into tab; xy (may be null): compact x/y rows; ztab (may be null): real z rows
static void launch_tab(const Grid& g, const FrameArg& fa, int qm_side, int with_ez, int max_n, const double* pos4,
                       int cap, double2* tab, double* ztab, double2* xy, hipStream_t s) {
  if (g.R <= kTabMaxR && 2 * g.mz <= kTabMaxZ) {
    // about kTabBlocks blocks in all, each looping over its frame's groups
    const int groups = (max_n + kTabAtoms - 1) / kTabAtoms;
    dim3 grid(std::max(1, std::min(groups, kTabBlocks / std::max(fa.n_frames, 1))), fa.n_frames);
    const size_t lds = (size_t)kTabAtoms * (g.NX + g.NY + (with_ez ? g.NZP : 0) + 1) * sizeof(double2);
    hipLaunchKernelGGL(k_prep_tab, grid, dim3(256), lds, s, g, fa, qm_side, with_ez, pos4, cap, tab, ztab, xy);
  } else {
    const long per = g.NX + g.NY + (with_ez ? g.NZP : 0) + (ztab ? g.mz : 0);
    dim3 grid((unsigned)(((long)max_n * per + 255) / 256), fa.n_frames);
    hipLaunchKernelGGL(k_prep_tab_direct, grid, dim3(256), 0, s, g, fa, qm_side, with_ez, pos4, cap, tab, ztab, xy);
  }
}

// ------------------------------------------------------------------ QM structure factors
// A(k) = sum_j Q_j e_j, B(k) = sum_j i (k.mu_j) e_j, C(k) = sum_j -1/2 (k.theta_j.k) e_j,
// e_j = e^{i k.R_j}  (SI, multipolar long-range tensors contracted with the moments).
// With with_w, also W(k) = (8 pi/V) g(k) S'(k) for the effective moments of the backward pass,
// and its folded form for the matrix-core adjoint: for column c and p = |nz| > 0,
// W+ = W(c, p), W- = W(c, -p), Ap = W+ + W-, Am = W+ - W-, so that
//   sum_nz W(c,nz) e^{-i nz kz0 z} = W(c,0) + sum_p [Ap cos(p kz0 z) - i Am sin(p kz0 z)]
//   sum_nz nz W(c,nz) e^{-i nz kz0 z} = sum_p p [Am cos(p kz0 z) - i Ap sin(p kz0 z)].
// Each thread owns one column and one p and evaluates both k = (nx, ny, +p) and (nx, ny, -p).
DEV void qm_terms(double (&v)[8], double2 e, double Qj, double kmu, double kthk) {
  v[0] += Qj * e.x;
  v[1] += Qj * e.y;
  v[2] -= kmu * e.y;
  v[3] += kmu * e.x;
  v[4] -= 0.5 * kthk * e.x;
  v[5] -= 0.5 * kthk * e.y;
}

__global__ __launch_bounds__(256) void k_sfac_qm(Grid g, FrameArg fa, const double* __restrict__ Q,
                                                 const double* __restrict__ mu, const double* __restrict__ theta,
                                                 const double* __restrict__ qeff, const double2* __restrict__ qtab,
                                                 int with_w, double2* __restrict__ sabc, double2* __restrict__ wk,
                                                 double* __restrict__ kw, double* __restrict__ wfrag,
                                                 double2* __restrict__ wk0) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int(threadIdx.x >> 6);
  const int NP = g.mz + 1;
  const int t = blockIdx.x * 64 + lane;
  const int tc = min(t, g.NCOL * NP - 1);
  const int col = tc / NP, p = tc - col * NP;
  const int nx = col / g.NY, iy = col - nx * g.NY;
  const int ny = iy - g.my;
  const double kx = 2.0 * kPi * nx * fr.inv_box[0], ky = 2.0 * kPi * ny * fr.inv_box[1],
               kz = 2.0 * kPi * p * fr.inv_box[2];
  double vp[8] = {0, 0, 0, 0, 0, 0, 0, 0}, vm[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // A, B, C, S' at +p and -p
  for (int j = wave; j < fr.nq; j += 4) {
    const int r = fr.qoff + j;
    const double2* row = qtab + (size_t)r * g.R;
    const double2 exy = cmul(row[nx], row[g.NX + iy]);
    const double2 ez = row[g.NX + g.NY + g.mz + p];
    const double2 ep = cmul(exy, ez), em = cmul(exy, cconj(ez));
    const double* m = mu + 3 * (size_t)r;
    const double* th = theta + 6 * (size_t)r;
    const double kmu_xy = kx * m[0] + ky * m[1], kmu_z = kz * m[2];
    const double kthk_xy = kx * kx * th[0] + ky * ky * th[3] + 2.0 * kx * ky * th[1];
    const double kthk_c = 2.0 * kz * (kx * th[2] + ky * th[4]), kthk_zz = kz * kz * th[5];
    const double Qj = Q[r];
    qm_terms(vp, ep, Qj, kmu_xy + kmu_z, kthk_xy + kthk_c + kthk_zz);
    qm_terms(vm, em, Qj, kmu_xy - kmu_z, kthk_xy - kthk_c + kthk_zz);
    if (with_w) {
      const double* qe = qeff + 10 * (size_t)r;
      const double emu_xy = kx * qe[1] + ky * qe[2], emu_z = kz * qe[3];
      const double eth_xy = kx * kx * qe[4] + ky * ky * qe[7] + 2.0 * kx * ky * qe[5];
      const double eth_c = 2.0 * kz * (kx * qe[6] + ky * qe[8]), eth_zz = kz * kz * qe[9];
      const double wrp = qe[0] - 0.5 * (eth_xy + eth_c + eth_zz), wip = emu_xy + emu_z;
      const double wrm = qe[0] - 0.5 * (eth_xy - eth_c + eth_zz), wim = emu_xy - emu_z;
      vp[6] += wrp * ep.x - wip * ep.y;
      vp[7] += wrp * ep.y + wip * ep.x;
      vm[6] += wrm * em.x - wim * em.y;
      vm[7] += wrm * em.y + wim * em.x;
    }
  }
  __shared__ double red[3][16][64];
  if (wave > 0)
    for (int u = 0; u < 8; u++) {
      red[wave - 1][u][lane] = vp[u];
      red[wave - 1][8 + u][lane] = vm[u];
    }
  __syncthreads();
  if (wave != 0 || t >= g.NCOL * NP) return;
  for (int u = 0; u < 8; u++) {
    vp[u] += red[0][u][lane] + red[1][u][lane] + red[2][u][lane];
    vm[u] += red[0][8 + u][lane] + red[1][8 + u][lane] + red[2][8 + u][lane];
  }
  const double V = fr.box[0] * fr.box[1] * fr.box[2];
  double2 W[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  for (int sg = 0; sg < 2; sg++) {
    if (sg == 1 && p == 0) break;
    const int nz = sg ? -p : p;
    const double* v = sg ? vm : vp;
    const int k = col * g.NZ + g.mz + nz;
    double2* o = sabc + ((size_t)f * g.KF + k) * 3;
    o[0] = make_double2(v[0], v[1]);
    o[1] = make_double2(v[2], v[3]);
    o[2] = make_double2(v[4], v[5]);
    double wgt = 0.0;
    if (in_half_space(nx, ny, nz)) {
      const double k2 = kx * kx + ky * ky + kz * kz;
      wgt = 8.0 * kPi / V * exp(-k2 / (4.0 * g.alpha * g.alpha)) / k2;
    }
    kw[(size_t)f * g.KF + k] = wgt;
    if (with_w) {
      W[sg] = make_double2(wgt * v[6], wgt * v[7]);
      wk[(size_t)f * g.KF + k] = W[sg];
    }
  }
  if (with_w && wfrag) {
    if (p == 0) {
      wk0[(size_t)f * g.NG * 16 + col] = W[0];
    } else {
      const double2 Ap = make_double2(W[0].x + W[1].x, W[0].y + W[1].y);
      const double2 Am = make_double2(W[0].x - W[1].x, W[0].y - W[1].y);
      const double fp = (double)p;
      // K row p-1 multiplies cos(p kz0 z), K row mz+p-1 multiplies sin(p kz0 z);
      // the four B matrices k = 0..3 give Re P, Im P, Re Pz, Im Pz.  A K step
      // holds 256 entries: entry 128 (k >> 1) + 2 lane + (k & 1) for lane =
      // column + 16 (K row & 3), so that a lane reads the B values of
      // matrices 0, 1 and of 2, 3 as two 16-byte loads
      double* base = wfrag + ((size_t)f * g.NG + (col >> 4)) * g.NK2 * 256 + 2 * (col & 15);
      double* o = base + (size_t)((p - 1) >> 2) * 256 + 32 * ((p - 1) & 3);
      o[0] = Ap.x;
      o[1] = Ap.y;
      o[128] = fp * Am.x;
      o[129] = fp * Am.y;
      const int js = g.mz + p - 1;
      o = base + (size_t)(js >> 2) * 256 + 32 * (js & 3);
      o[0] = Am.y;
      o[1] = -Am.x;
      o[128] = fp * Ap.y;
      o[129] = -fp * Ap.x;
    }
  }
}

hipError_t launch_sfac_qm(const Grid& g, const FrameArg& fa, int max_nq, const double* Q, const double* mu,
                          const double* theta, const double* qeff, const double* gE, int with_w, Work& w,
                          hipStream_t s) {
  (void)max_nq;
  (void)gE;
  dim3 grid((g.NCOL * (g.mz + 1) + 63) / 64, fa.n_frames);
  hipLaunchKernelGGL(k_sfac_qm, grid, dim3(256), 0, s, g, fa, Q, mu, theta, qeff, w.qm_tab, with_w, w.sabc, w.wk,
                     w.kw, w.wfrag, w.wk0);
  if (with_w && w.wfrag32) return launch_wfrag32(g, fa, w, s);
  return hipGetLastError();
}

// v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16).  A[i][k] sits in lane
// i + 16k, B[k][j] in lane j + 16k, and element r of D in lane l is D[l/16 + 4r][l%16].
typedef double v4d __attribute__((ext_vector_type(4)));

DEV v4d mfma4(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Raw buffer loads: a resource holds a wave-uniform base and a byte count
// (loads past it return zero without touching memory); the offset is a
// per-lane byte offset plus a uniform (scalar) byte offset.
DEV __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
DEV double buf_load_f64(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
DEV double2 buf_load_c64(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// ------------------------------------------------------------------ MM structure factor (forward hot loop)
// S_MM(k) = sum_i q_i e^{i k.R_i}.  Each lane owns one column (nx,ny) and Z
// consecutive nz values; for every atom it forms c = q e^{i(kx x + ky y)}
// from the atom's table row and accumulates c * e^{i kz z} with four FMAs per
// k, the z phases being wave-uniform (scalar loads).  The four waves of a
// block split the block's atom range and are summed through LDS; the block
// writes one partial sum per k, and partial sums over atom chunks are added
// by k_reduce_smm.
template <int Z, bool PF>
__global__ __launch_bounds__(256) void k_sfac_mm(Grid g, FrameArg fa, int a_chunk, int nkb, int nac,
                                                 const double* __restrict__ mm4, int cap_mm,
                                                 const double2* __restrict__ tab, double2* __restrict__ spart) {
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  const int kb = blockIdx.x % nkb, ac = blockIdx.x / nkb;
  if (ac >= nac) return;
  const int nzc = g.NZP / Z;
  const int tile = kb / nzc, zc = kb - tile * nzc;
  const int a0 = ac * a_chunk;
  if (a0 >= fr.nm || tile * 64 >= g.NCOL) return;
  const int a1 = min(fr.nm, a0 + a_chunk);
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int(threadIdx.x >> 6);
  const int col = tile * 64 + lane;
  const int colc = min(col, g.NCOL - 1);
  const int nx = colc / g.NY, iy = colc - nx * g.NY;

  double sr[Z], si[Z];
#pragma unroll
  for (int z = 0; z < Z; z++) {
    sr[z] = 0.0;
    si[z] = 0.0;
  }
  const double* __restrict__ qv = mm4 + (size_t)3 * cap_mm + fr.moff;
  const double2* __restrict__ base = tab + (size_t)fr.moff * g.R;
  const int zoff = g.NX + g.NY + zc * Z;
  int a = a0 + wave;
  // optional software pipeline: the lane-specific factors of the next atom are
  // in flight while the current atom is accumulated
  double qn = 0.0;
  double2 exn = make_double2(0, 0), eyn = make_double2(0, 0);
  if (PF && a < a1) {
    const double2* __restrict__ row = base + (size_t)a * g.R;
    qn = qv[a];
    exn = row[nx];
    eyn = row[g.NX + iy];
  }
  for (; a < a1; a += 4) {
    double q;
    double2 ex, ey;
    if (PF) {
      q = qn;
      ex = exn;
      ey = eyn;
      const int an = a + 4;
      if (an < a1) {
        const double2* __restrict__ rown = base + (size_t)an * g.R;
        qn = qv[an];
        exn = rown[nx];
        eyn = rown[g.NX + iy];
      }
    } else {
      const double2* __restrict__ rowc = base + (size_t)a * g.R;
      q = qv[a];
      ex = rowc[nx];
      ey = rowc[g.NX + iy];
    }
    const double cr = q * (ex.x * ey.x - ex.y * ey.y);
    const double ci = q * (ex.x * ey.y + ex.y * ey.x);
    const double2* __restrict__ ez = base + (size_t)a * g.R + zoff;
#pragma unroll
    for (int z = 0; z < Z; z++) {
      const double2 e = ez[z];
      sr[z] = fma(cr, e.x, sr[z]);
      sr[z] = fma(-ci, e.y, sr[z]);
      si[z] = fma(cr, e.y, si[z]);
      si[z] = fma(ci, e.x, si[z]);
    }
  }
  // combine the four waves: 3,2 -> 1,0 -> 0
  __shared__ double2 red[2][Z][64];
  if (wave >= 2) {
#pragma unroll
    for (int z = 0; z < Z; z++) red[wave - 2][z][lane] = make_double2(sr[z], si[z]);
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int z = 0; z < Z; z++) {
      const double2 o = red[wave][z][lane];
      sr[z] += o.x;
      si[z] += o.y;
    }
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int z = 0; z < Z; z++) red[0][z][lane] = make_double2(sr[z], si[z]);
  }
  __syncthreads();
  if (wave == 0 && col < g.NCOL) {
    double2* __restrict__ out = spart + (size_t)(fr.slot_base + ac) * g.NZP * g.NCOL;
#pragma unroll
    for (int z = 0; z < Z; z++) {
      const double2 o = red[0][z][lane];
      out[(size_t)(zc * Z + z) * g.NCOL + col] = make_double2(sr[z] + o.x, si[z] + o.y);
    }
  }
}

bool sfac_mm_has_zc(int zc) {
  switch (zc) {
    case 7: case 8: case 11: case 12: case 13: case 14: case 16: case 17: case 21: case 25:
      return true;
    default:
      return false;
  }
}

// nz chunk with the least padding, preferring larger chunks on ties
int pick_zc(int NZ) {
  static const int cands[] = {25, 21, 17, 16, 14, 13, 12, 11};
  int best = 17;
  double best_cost = 1e30;
  for (int c : cands) {
    const int nzc = (NZ + c - 1) / c;
    const double waste = (double)(nzc * c - NZ) / NZ;
    // per-atom overhead of forming c is about 6 FMA-equivalents per lane
    const double cost = (1.0 + waste) * (1.0 + 6.0 / (4.0 * c));
    if (cost < best_cost - 1e-12) {
      best_cost = cost;
      best = c;
    }
  }
  return best;
}

template <int Z>
static hipError_t launch_sfac_mm_z(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm,
                                   Work& w, hipStream_t s) {
  const int tiles = (g.NCOL + 63) / 64;
  const int nkb = tiles * (g.NZP / Z);
  const int nac = (max_nm + t.a_chunk - 1) / t.a_chunk;
  if (nac == 0) return hipSuccess;
  dim3 grid(nkb * nac, 1, fa.n_frames);
  if (t.fwd_pf)
    hipLaunchKernelGGL((k_sfac_mm<Z, true>), grid, dim3(256), 0, s, g, fa, t.a_chunk, nkb, nac, w.mm4, cap_mm, w.mm_tab,
                       w.spart);
  else
    hipLaunchKernelGGL((k_sfac_mm<Z, false>), grid, dim3(256), 0, s, g, fa, t.a_chunk, nkb, nac, w.mm4, cap_mm,
                       w.mm_tab, w.spart);
  return hipGetLastError();
}

static hipError_t launch_sfac_mm_mfma(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm,
                                      Work& w, hipStream_t s);

hipError_t launch_sfac_mm(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                          hipStream_t s) {
  if (t.fp32r) return launch_sfac_mm32(g, t, fa, max_nm, cap_mm, w, s);
  if (t.fwd_mode == 1) {
    if (!tab32_ok(g, max_nm)) return hipErrorInvalidValue;  // the API rejects such frames first
    return launch_sfac_mm_mfma(g, t, fa, max_nm, cap_mm, w, s);
  }
  switch (g.Zc) {
    case 7: return launch_sfac_mm_z<7>(g, t, fa, max_nm, cap_mm, w, s);
    case 8: return launch_sfac_mm_z<8>(g, t, fa, max_nm, cap_mm, w, s);
    case 11: return launch_sfac_mm_z<11>(g, t, fa, max_nm, cap_mm, w, s);
    case 12: return launch_sfac_mm_z<12>(g, t, fa, max_nm, cap_mm, w, s);
    case 13: return launch_sfac_mm_z<13>(g, t, fa, max_nm, cap_mm, w, s);
    case 14: return launch_sfac_mm_z<14>(g, t, fa, max_nm, cap_mm, w, s);
    case 16: return launch_sfac_mm_z<16>(g, t, fa, max_nm, cap_mm, w, s);
    case 17: return launch_sfac_mm_z<17>(g, t, fa, max_nm, cap_mm, w, s);
    case 21: return launch_sfac_mm_z<21>(g, t, fa, max_nm, cap_mm, w, s);
    case 25: return launch_sfac_mm_z<25>(g, t, fa, max_nm, cap_mm, w, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------ matrix-core forward
// The z phases of +p and -p are complex conjugates, so with
//   C_i(c) = q_i e^{i(kx x_i + ky y_i)}                   (column c = (nx, ny))
//   U(c,p) = sum_i C_i(c) cos(p kz0 z_i),  V(c,p) = sum_i C_i(c) sin(p kz0 z_i)
// the structure factor is S(c, +p) = U + iV, S(c, -p) = U - iV, S(c, 0) = sum_i C_i(c).
// U and V are one real contraction over atoms: [Re C; Im C] (columns x atoms)
// times the real z table (atoms x [cos | sin]), done on the FP64 matrix cores
// with 4 atoms per K step.  A block of four waves covers CT 16-column tiles
// and one atom chunk (the waves interleave its K steps); the waves are summed
// through LDS and the block writes one partial S per k in k order.
// LDS doubles of one forward item: two wave-pair accumulator sets, and the
// nz = 0 sums of the four waves
template <int CT, int NT>
constexpr int sfac_lds_doubles() {
  return 2 * CT * NT * 8 * 64 + 4 * CT * 2 * 16;
}

// One forward work item: column group gc (CT 16-column tiles) of atom chunk ac
// of frame fr, all 256 threads of the block; lds holds sfac_lds_doubles().
// Returns (uniformly) for a chunk past the frame's atoms.
template <int CT, int NT>
DEV void sfac_mm_mfma_item(const Grid& g, const FrameDev& fr, int gc, int ac, int a_chunk,
                           const double* __restrict__ mm4, int cap_mm, const double2* __restrict__ tab,
                           const double* __restrict__ ztab, double2* __restrict__ spart, double* lds) {
  static_assert(CT * NT <= 8, "LDS budget of the block reduction (66 KB at 8)");
  constexpr int NACC = CT * NT * 8;  // accumulator doubles per lane
  double* red[2] = {lds, lds + NACC * 64};
  double(*s0red)[CT][2][16] = reinterpret_cast<double(*)[CT][2][16]>(lds + 2 * NACC * 64);
  const int a0 = ac * a_chunk;
  if (a0 >= fr.nm) return;  // uniform over the block
  const int a1 = min(fr.nm, a0 + a_chunk);
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  int cx[CT], cy[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    const int col = min((gc * CT + ct) * 16 + li, g.NCOL - 1);
    const int nx = col / g.NY;
    cx[ct] = nx;
    cy[ct] = g.NX + col - nx * g.NY;
  }
  v4d dr[CT][NT], di[CT][NT];
  double s0r[CT], s0i[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    s0r[ct] = s0i[ct] = 0.0;
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
      dr[ct][nt] = v4d{0.0, 0.0, 0.0, 0.0};
      di[ct][nt] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  }
  // Operands are buffer loads from resources that end at the chunk's last
  // atom (rows past it read as zero, so a partial K step needs no clamp or
  // select), with one offset per lane and a uniform offset per K step.  The
  // loads of step i + 1 are issued before step i is contracted; two steps are
  // unrolled so that the prefetched operands need no register copies, and the
  // order is fixed with scheduling barriers (the compiler would otherwise
  // move the loads next to their use).  Lane: column li of each tile, atom
  // a + lk of the step (row k of B and column k of A).
  const int arow = a0 + 4 * wave + lk;
  const __amdgpu_buffer_rsrc_t qr = buf_rsrc(mm4 + (size_t)3 * cap_mm + fr.moff, (unsigned)a1 * 8u);
  const __amdgpu_buffer_rsrc_t tr = buf_rsrc(tab + (size_t)fr.moff * g.NXY, (unsigned)a1 * g.NXY * 16u);
  const __amdgpu_buffer_rsrc_t zr = buf_rsrc(ztab + (size_t)fr.moff * g.ZKP, (unsigned)a1 * g.ZKP * 8u);
  const int qo = arow * 8, zo = (arow * g.ZKP + li) * 8;
  int xo[CT], yo[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    xo[ct] = (arow * g.NXY + cx[ct]) * 16;
    yo[ct] = (arow * g.NXY + cy[ct]) * 16;
  }
  const int ts = 16 * g.NXY * 16, zs = 16 * g.ZKP * 8;  // bytes per K step (16 atoms)
  const int nst = a0 + 4 * wave < a1 ? (a1 - a0 - 4 * wave + 15) / 16 : 0;
  struct Ops {
    double q;
    double2 ex[CT], ey[CT];
    double bz[NT];
  };
  auto fetch = [&](int i, Ops& o) {
    o.q = buf_load_f64(qr, qo, i * 128);
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      o.ex[ct] = buf_load_c64(tr, xo[ct], i * ts);
      o.ey[ct] = buf_load_c64(tr, yo[ct], i * ts);
    }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) o.bz[nt] = buf_load_f64(zr, zo + nt * 128, i * zs);
  };
  auto step = [&](const Ops& o) {
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      const double pr = fma(o.ex[ct].x, o.ey[ct].x, -o.ex[ct].y * o.ey[ct].y);
      const double pi = fma(o.ex[ct].x, o.ey[ct].y, o.ex[ct].y * o.ey[ct].x);
      const double cr = o.q * pr, ci = o.q * pi;
      s0r[ct] += cr;
      s0i[ct] += ci;
#pragma unroll
      for (int nt = 0; nt < NT; nt++) {
        dr[ct][nt] = mfma4(cr, o.bz[nt], dr[ct][nt]);
        di[ct][nt] = mfma4(ci, o.bz[nt], di[ct][nt]);
      }
    }
  };
  // (a fetch past the last step reads rows past the chunk: zeros)
  Ops A, B;
  fetch(0, A);
  int i = 0;
  for (; i + 1 < nst; i += 2) {
    __builtin_amdgcn_sched_barrier(0);
    fetch(i + 1, B);
    __builtin_amdgcn_sched_barrier(0);
    step(A);
    __builtin_amdgcn_sched_barrier(0);
    fetch(i + 2, A);
    __builtin_amdgcn_sched_barrier(0);
    step(B);
  }
  if (i < nst) step(A);
  // nz = 0: sum over the four atom rows of the wave, then over the waves
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    s0r[ct] += __shfl_xor(s0r[ct], 16, 64);
    s0r[ct] += __shfl_xor(s0r[ct], 32, 64);
    s0i[ct] += __shfl_xor(s0i[ct], 16, 64);
    s0i[ct] += __shfl_xor(s0i[ct], 32, 64);
    if (lk == 0) {
      s0red[wave][ct][0][li] = s0r[ct];
      s0red[wave][ct][1][li] = s0i[ct];
    }
  }
  // waves 3,2 -> 1,0 -> 0
  auto store = [&](double* dst) {
    int idx = 0;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int nt = 0; nt < NT; nt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          dst[(idx++) * 64 + lane] = dr[ct][nt][r];
          dst[(idx++) * 64 + lane] = di[ct][nt][r];
        }
  };
  auto add = [&](const double* src) {
    int idx = 0;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int nt = 0; nt < NT; nt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          dr[ct][nt][r] += src[(idx++) * 64 + lane];
          di[ct][nt][r] += src[(idx++) * 64 + lane];
        }
  };
  if (wave >= 2) store(red[wave - 2]);
  __syncthreads();
  if (wave < 2) add(red[wave]);
  __syncthreads();
  if (wave == 1) store(red[0]);
  __syncthreads();
  constexpr int NCL = CT * 16, NJ = NT * 16;
  double* T = red[1];  // T[0][c][j] = U/V real parts, T[1][c][j] = imaginary parts
  if (wave == 0) {
    add(red[0]);
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int nt = 0; nt < NT; nt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int c = ct * 16 + lk + 4 * r, j = nt * 16 + li;
          T[c * NJ + j] = dr[ct][nt][r];
          T[(NCL + c) * NJ + j] = di[ct][nt][r];
        }
  }
  __syncthreads();
  double2* __restrict__ out = spart + (size_t)(fr.slot_base + ac) * g.NZP * g.NCOL;
  // entry e = c NZ + iz; (c, iz) advance by the block size without a division
  // per entry (c grows with e, so the first column past the grid ends the loop)
  const int dc = 256 / g.NZ, diz = 256 - dc * g.NZ;
  int c = threadIdx.x / g.NZ, iz = threadIdx.x - c * g.NZ;
  for (int e = threadIdx.x; e < NCL * g.NZ; e += 256, c += dc, iz += diz) {
    if (iz >= g.NZ) {
      iz -= g.NZ;
      c++;
    }
    const int col = gc * NCL + c;
    if (col >= g.NCOL) break;
    const int nz = iz - g.mz;
    double2 S;
    if (nz == 0) {
      const int ct = c >> 4, cl = c & 15;
      S.x = ((s0red[0][ct][0][cl] + s0red[1][ct][0][cl]) + s0red[2][ct][0][cl]) + s0red[3][ct][0][cl];
      S.y = ((s0red[0][ct][1][cl] + s0red[1][ct][1][cl]) + s0red[2][ct][1][cl]) + s0red[3][ct][1][cl];
    } else {
      const int pj = (nz > 0 ? nz : -nz) - 1;
      const double ur = T[c * NJ + pj], ui = T[(NCL + c) * NJ + pj];
      const double vr = T[c * NJ + g.mz + pj], vi = T[(NCL + c) * NJ + g.mz + pj];
      S = nz > 0 ? make_double2(ur - vi, ui + vr) : make_double2(ur + vi, ui - vr);
    }
    out[(size_t)col * g.NZ + iz] = S;
  }
}

template <int CT, int NT>
__global__ __launch_bounds__(256) void k_sfac_mm_mfma(Grid g, FrameArg fa, int a_chunk, int ngc, int nac,
                                                      int xcd_remap, int units, const double* __restrict__ mm4,
                                                      int cap_mm, const double2* __restrict__ tab,
                                                      const double* __restrict__ ztab,
                                                      double2* __restrict__ spart) {
  __shared__ double lds[sfac_lds_doubles<CT, NT>()];
  // Consecutive workgroups go to the 8 XCDs in turn.  Many frames: the
  // XCD-aware order over (frame, atom chunk) units, whose blocks then share
  // their atom rows in one XCD's L2 (largest frames first, so that the snake
  // order gives each XCD a similar share).
  if (units > 0) {
    int f, gc, ac;
    if (!fwd_unit(fa, units, ngc, f, gc, ac)) return;
    const FrameDev fr = get_frame(fa, f);
    if (ac < 0 || ac * a_chunk >= fr.nm) return;
    sfac_mm_mfma_item<CT, NT>(g, fr, gc, ac, a_chunk, mm4, cap_mm, tab, ztab, spart, lds);
    return;
  }
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  // With xcd_remap (single frame) the blocks that share an atom chunk
  // (consecutive logical ids) are placed on one XCD, so that its L2 serves
  // their common atom rows.
  int bid = blockIdx.x;
  if (xcd_remap) {
    const int per = (int)gridDim.x / 8;
    if (bid < 8 * per) bid = (bid % 8) * per + bid / 8;
  }
  const int gc = bid % ngc, ac = bid / ngc;
  if (ac >= nac) return;
  sfac_mm_mfma_item<CT, NT>(g, fr, gc, ac, a_chunk, mm4, cap_mm, tab, ztab, spart, lds);
}

template <int CT, int NT>
static void launch_sfac_mm_mfma_t(dim3 grid, hipStream_t s, const Grid& g, const FrameArg& fa, int a_chunk, int ngc,
                                  int nac, int xcd, int units, int cap_mm, Work& w) {
  hipLaunchKernelGGL((k_sfac_mm_mfma<CT, NT>), grid, dim3(256), 0, s, g, fa, a_chunk, ngc, nac, xcd, units, w.mm4,
                     cap_mm, w.mm_xy, w.mm_ztab, w.spart);
}

static hipError_t launch_sfac_mm_mfma(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm,
                                      Work& w, hipStream_t s) {
  const int ngc = fwd_col_groups(g, t);
  const int nac = (max_nm + t.a_chunk - 1) / t.a_chunk;
  if (nac == 0) return hipSuccess;
  dim3 grid(ngc * nac, 1, fa.n_frames);
  const int xcd = (t.fwd_xcd && fa.n_frames == 1) ? 1 : 0;
  // many frames: one-dimensional grid over the partial-sum slots (units)
  const int units = (t.fwd_xcd && fa.frames && fa.n_frames > 1) ? t.fwd_units : 0;
  if (units > 0) grid = dim3(8 * ngc * ((units + 7) / 8), 1, 1);
#define SF(C, N)                                                                             \
  if (t.fwd_ct == C && g.NT == N) {                                                          \
    launch_sfac_mm_mfma_t<C, N>(grid, s, g, fa, t.a_chunk, ngc, nac, xcd, units, cap_mm, w); \
    return hipGetLastError();                                                                \
  }
  SF(1, 1) SF(2, 1) SF(4, 1) SF(1, 2) SF(2, 2) SF(4, 2) SF(1, 3) SF(2, 3) SF(1, 4) SF(2, 4)
#undef SF
  return hipErrorInvalidValue;
}

// Reference GPU path: one thread per k, sincos of k.R for every atom.
__global__ __launch_bounds__(256) void k_sfac_mm_plain(Grid g, FrameArg fa, const double* __restrict__ mm4,
                                                       int cap_mm, double2* __restrict__ spart) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int e = blockIdx.x * 256 + threadIdx.x;  // e = iz * NCOL + col
  if (e >= g.NZ * g.NCOL) return;
  const int iz = e / g.NCOL, col = e - iz * g.NCOL;
  const int nx = col / g.NY, iy = col - nx * g.NY;
  const double kx = 2.0 * kPi * nx * fr.inv_box[0], ky = 2.0 * kPi * (iy - g.my) * fr.inv_box[1],
               kz = 2.0 * kPi * (iz - g.mz) * fr.inv_box[2];
  double sr = 0.0, si = 0.0;
  const double* x = mm4 + fr.moff;
  const double* y = mm4 + (size_t)cap_mm + fr.moff;
  const double* z = mm4 + (size_t)2 * cap_mm + fr.moff;
  const double* q = mm4 + (size_t)3 * cap_mm + fr.moff;
  for (int i = 0; i < fr.nm; i++) {
    double sn, cs;
    sincos(kx * x[i] + ky * y[i] + kz * z[i], &sn, &cs);
    sr += q[i] * cs;
    si += q[i] * sn;
  }
  spart[(size_t)fr.slot_base * g.NZP * g.NCOL + (size_t)iz * g.NCOL + col] = make_double2(sr, si);
}

hipError_t launch_sfac_mm_plain(const Grid& g, const FrameArg& fa, int cap_mm, Work& w, hipStream_t s) {
  dim3 grid((g.NZ * g.NCOL + 255) / 256, fa.n_frames);
  hipLaunchKernelGGL(k_sfac_mm_plain, grid, dim3(256), 0, s, g, fa, w.mm4, cap_mm, w.spart);
  return hipGetLastError();
}

// Sum the partial structure factors, store S_MM in k order, and accumulate
// the reciprocal energies (8 pi/V) g Re[S_QM conj S_MM] and the order-2
// truncated QM-QM term (4 pi/V) g (|A|^2 + 2Re A*B + 2Re A*C + |B|^2).
// Partial sums are in k order (kmajor, matrix-core forward) or nz-major
// (VALU and plain forward).
// One item: the 256 reciprocal vectors of block kb (of nkb) of frame f; red
// holds 8 doubles of LDS.
DEV void reduce_smm_item(const Grid& g, const FrameDev& fr, int f, int kb, int nkb, int a_chunk, int plain,
                         int kmajor, const double2* __restrict__ spart, const double2* __restrict__ sabc,
                         const double* __restrict__ kw, double2* __restrict__ smm, size_t smm_stride,
                         double* __restrict__ facc, double* __restrict__ det, double* red) {
  const int k = kb * 256 + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (k < g.KF) {
    const int col = k / g.NZ, iz = k - col * g.NZ;
    const int nslots = plain ? 1 : (fr.nm + a_chunk - 1) / a_chunk;
    const size_t idx = kmajor ? (size_t)k : (size_t)iz * g.NCOL + col;
    // eight partials in flight per round trip (a load-add chain per slot left
    // the kernel latency bound); the slots are still summed in order
    const size_t sstride = (size_t)g.NZP * g.NCOL;
    const double2* __restrict__ pp = spart + (size_t)fr.slot_base * sstride + idx;
    double sr = 0.0, si = 0.0;
    int sl = 0;
    for (; sl + 8 <= nslots; sl += 8) {
      double2 p[8];
#pragma unroll
      for (int u = 0; u < 8; u++) p[u] = pp[(size_t)(sl + u) * sstride];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        sr += p[u].x;
        si += p[u].y;
      }
    }
    for (; sl < nslots; sl++) {
      const double2 p = pp[(size_t)sl * sstride];
      sr += p.x;
      si += p.y;
    }
    if (plain && fr.nm == 0) sr = si = 0.0;
    smm[(size_t)f * smm_stride + k] = make_double2(sr, si);
    const double wgt = kw[(size_t)f * g.KF + k];
    if (wgt != 0.0) {
      const double2* abc = sabc + ((size_t)f * g.KF + k) * 3;
      const double2 A = abc[0], B = abc[1], C = abc[2];
      const double sqr = A.x + B.x + C.x, sqi = A.y + B.y + C.y;
      v[0] = wgt * (sqr * sr + sqi * si);
      const double F = (A.x * A.x + A.y * A.y) + 2.0 * (A.x * B.x + A.y * B.y) + 2.0 * (A.x * C.x + A.y * C.y) +
                       (B.x * B.x + B.y * B.y);
      v[1] = 0.5 * wgt * F;
    }
  }
  double tot[2];
  block_sum256_lds<2>(v, tot, red);
  if (threadIdx.x == 0) {
    if (det) {
      double* o = det + ((size_t)f * nkb + kb) * 2;
      o[0] = tot[0];
      o[1] = tot[1];
    } else {
      atomicAdd(&facc[f * FA_COUNT + FA_E_QMMM_LR], tot[0]);
      atomicAdd(&facc[f * FA_COUNT + FA_E_QQ_LR], tot[1]);
    }
  }
}

__global__ __launch_bounds__(256) void k_reduce_smm(Grid g, FrameArg fa, int a_chunk, int plain, int kmajor,
                                                    const double2* __restrict__ spart,
                                                    const double2* __restrict__ sabc,
                                                    const double* __restrict__ kw, double2* __restrict__ smm,
                                                    size_t smm_stride, double* __restrict__ facc,
                                                    double* __restrict__ det) {
  __shared__ double red[8];
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  reduce_smm_item(g, fr, f, blockIdx.x, gridDim.x, a_chunk, plain, kmajor, spart, sabc, kw, smm, smm_stride, facc,
                  det, red);
}

hipError_t launch_reduce_smm(const Grid& g, const Tuning& t, const FrameArg& fa, int plain, double2* smm_out,
                             size_t smm_frame_stride, Work& w, hipStream_t s) {
  dim3 grid((g.KF + 255) / 256, fa.n_frames);
  const int kmajor = !plain && t.fwd_mode == 1;
  hipLaunchKernelGGL(k_reduce_smm, grid, dim3(256), 0, s, g, fa, t.a_chunk, plain, kmajor, w.spart, w.sabc, w.kw,
                     smm_out, smm_frame_stride, w.facc, w.det_smm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !w.det_smm) return e;
  return launch_det_reduce(fa, 0, 1, w.det_smm, (int)grid.x, 2, det_map({FA_E_QMMM_LR, FA_E_QQ_LR}), w.facc,
                           FA_COUNT, s);
}

// ------------------------------------------------------------------ QM-site projection
// Forward: phi, grad phi and 1/2 grad grad phi of the MM charges at each QM
// site from S_MM.  Backward: the QM-MM long-range gradient with the
// effective moments, and the QM-QM long-range gradient and moment
// derivatives of the order-2 truncated image energy.
// LDS doubles of the projection's block sums
template <int BWD>
constexpr int project_lds_doubles() {
  return 4 * (BWD == 0 ? 10 : BWD == 1 ? 16 : 26);
}

// One item: sites sb S .. sb S + S - 1 of frame f, the k items of block pc of
// n_pc; red holds project_lds_doubles<BWD>().
template <int BWD, int S>
DEV void project_qm_item(const Grid& g, const FrameDev& fr, int f, int sb, int pc, int n_pc,
                         const double2* __restrict__ smm, size_t smm_stride, const double* __restrict__ Q,
                         const double* __restrict__ mu, const double* __restrict__ theta,
                         const double* __restrict__ qeff, const double2* __restrict__ qtab,
                         const double2* __restrict__ sabc, const double* __restrict__ kw, int qmqm,
                         double* __restrict__ qacc, double* __restrict__ det, double* red) {
  // S sites per block: the per-k data (weight, S_MM, A/B/C) is loaded once per
  // k and applied to each site; the sites' moments are block-uniform
  const int j0 = sb * S;
  if (j0 >= fr.nq) return;
  const int ns = min(S, fr.nq - j0);  // uniform
  // BWD: 0 forward (10 sums), 1 adjoint (16), 2 both (26, adjoint after the forward ones)
  constexpr int NV = BWD == 0 ? 10 : BWD == 1 ? 16 : 26;
  constexpr int OB = BWD == 2 ? 10 : 0;
  double acc[S][NV];
#pragma unroll
  for (int u = 0; u < S; u++)
#pragma unroll
    for (int t = 0; t < NV; t++) acc[u][t] = 0.0;
  struct Mom {
    double Qe, m0, m1, m2, t0, t1, t2, t3, t4, t5, Qo, o0, o1, o2, u0, u1, u2, u3, u4, u5;
  };
  Mom mo[S];
  const double2* row[S];
#pragma unroll
  for (int u = 0; u < S; u++) {
    const int r = fr.qoff + min(j0 + u, fr.nq - 1);
    row[u] = qtab + (size_t)r * g.R;
    Mom& m = mo[u];
    m = Mom{};
    if (BWD) {
      const double* qe = qeff + 10 * (size_t)r;
      m.Qe = qe[0]; m.m0 = qe[1]; m.m1 = qe[2]; m.m2 = qe[3];
      m.t0 = qe[4]; m.t1 = qe[5]; m.t2 = qe[6]; m.t3 = qe[7]; m.t4 = qe[8]; m.t5 = qe[9];
      m.Qo = Q[r]; m.o0 = mu[3 * (size_t)r]; m.o1 = mu[3 * (size_t)r + 1]; m.o2 = mu[3 * (size_t)r + 2];
      const double* th = theta + 6 * (size_t)r;
      m.u0 = th[0]; m.u1 = th[1]; m.u2 = th[2]; m.u3 = th[3]; m.u4 = th[4]; m.u5 = th[5];
    }
  }
  // thread item = (column, p = |nz|): k = (nx, ny, +p) and (nx, ny, -p) share e^{i(kx x + ky y)}
  const int NP = g.mz + 1;
  const int n_items = g.NCOL * NP;
  for (int t = pc * 256 + threadIdx.x; t < n_items; t += n_pc * 256) {
    const int col = t / NP, p = t - col * NP;
    const int nx = col / g.NY, iy = col - nx * g.NY;
    const int ny = iy - g.my;
    double2 exy[S], ez[S];
#pragma unroll
    for (int u = 0; u < S; u++) {
      exy[u] = cmul(row[u][nx], row[u][g.NX + iy]);
      ez[u] = row[u][g.NX + g.NY + g.mz + p];
    }
    // both signs of nz at once, without data-dependent branches, so that all
    // the item's loads are issued together (one round trip per item); the
    // second sign of p = 0 and k outside the half space carry zero weight
    const int k0 = col * g.NZ + g.mz;
    double wv[2];
    double2 Sv[2], Av[2], Bv[2], Cv[2];
#pragma unroll
    for (int sg = 0; sg < 2; sg++) {
      const int k = k0 + (sg ? -p : p);
      wv[sg] = (sg && p == 0) ? 0.0 : kw[(size_t)f * g.KF + k];
      Sv[sg] = smm[(size_t)f * smm_stride + k];
      Av[sg] = Bv[sg] = Cv[sg] = make_double2(0.0, 0.0);
      if (BWD != 0 && qmqm) {
        const double2* abc = sabc + ((size_t)f * g.KF + k) * 3;
        Av[sg] = abc[0];
        Bv[sg] = abc[1];
        Cv[sg] = abc[2];
      }
    }
#pragma unroll
    for (int sg = 0; sg < 2; sg++) {
      const int nz = sg ? -p : p;
      const double w = wv[sg];
      const double kx = 2.0 * kPi * nx * fr.inv_box[0], ky = 2.0 * kPi * ny * fr.inv_box[1],
                   kz = 2.0 * kPi * nz * fr.inv_box[2];
      const double2 Sk = Sv[sg], A = Av[sg], B = Bv[sg], C = Cv[sg];
#pragma unroll
      for (int u = 0; u < S; u++) {
        if (u >= ns) break;  // uniform
        const Mom& m = mo[u];
        double* ac = acc[u];
        const double2 e = cmul(exy[u], sg ? cconj(ez[u]) : ez[u]);
        // Y = e conj(S)
        const double yr = e.x * Sk.x + e.y * Sk.y, yi = e.y * Sk.x - e.x * Sk.y;
        if (BWD != 1) {
          ac[0] += w * yr;
          ac[1] -= w * kx * yi;
          ac[2] -= w * ky * yi;
          ac[3] -= w * kz * yi;
          const double h = -0.5 * w * yr;
          ac[4] += h * kx * kx;
          ac[5] += h * kx * ky;
          ac[6] += h * kx * kz;
          ac[7] += h * ky * ky;
          ac[8] += h * ky * kz;
          ac[9] += h * kz * kz;
        }
        if (BWD != 0) {
          // QM-MM: d/dR of Re[(Q' + i k.mu' - 1/2 k.th'.k) Y] = k Re[i (..) Y]
          const double kthk = kx * kx * m.t0 + ky * ky * m.t3 + kz * kz * m.t5 +
                              2.0 * (kx * ky * m.t1 + kx * kz * m.t2 + ky * kz * m.t4);
          const double wr = m.Qe - 0.5 * kthk, wi = kx * m.m0 + ky * m.m1 + kz * m.m2;
          const double gr = -(wr * yi + wi * yr);
          ac[OB + 0] += w * kx * gr;
          ac[OB + 1] += w * ky * gr;
          ac[OB + 2] += w * kz * gr;
          if (qmqm) {
            const double kmu = kx * m.o0 + ky * m.o1 + kz * m.o2;
            const double kthko = kx * kx * m.u0 + ky * ky * m.u3 + kz * kz * m.u5 +
                                 2.0 * (kx * ky * m.u1 + kx * kz * m.u2 + ky * kz * m.u4);
            // a_j = Q e, b_j = i kmu e, c_j = -1/2 kthk e
            const double ajr = m.Qo * e.x, aji = m.Qo * e.y;
            const double bjr = -kmu * e.y, bji = kmu * e.x;
            const double cjr = -0.5 * kthko * e.x, cji = -0.5 * kthko * e.y;
            const double T1r = A.x + B.x + C.x, T1i = A.y + B.y + C.y;
            const double T2r = A.x + B.x, T2i = A.y + B.y;
            // Im[a_j conj(T1) + b_j conj(T2) + c_j conj(A)]
            const double zi = (aji * T1r - ajr * T1i) + (bji * T2r - bjr * T2i) + (cji * A.x - cjr * A.y);
            ac[OB + 3] -= w * kx * zi;
            ac[OB + 4] -= w * ky * zi;
            ac[OB + 5] -= w * kz * zi;
            ac[OB + 6] += w * (e.x * T1r + e.y * T1i);
            const double ime = e.y * T2r - e.x * T2i;
            ac[OB + 7] -= w * kx * ime;
            ac[OB + 8] -= w * ky * ime;
            ac[OB + 9] -= w * kz * ime;
            const double h = -0.5 * w * (e.x * A.x + e.y * A.y);
            ac[OB + 10] += h * kx * kx;
            ac[OB + 11] += h * kx * ky;
            ac[OB + 12] += h * kx * kz;
            ac[OB + 13] += h * ky * ky;
            ac[OB + 14] += h * ky * kz;
            ac[OB + 15] += h * kz * kz;
          }
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < S; u++) {
    if (u >= ns) break;  // uniform
    double tot[NV];
    block_sum256_lds<NV>(acc[u], tot, red);
    if (threadIdx.x == 0 && det) {
      // partial sums of this block, summed over the blocks in order afterwards
      double* o = det + ((size_t)(fr.qoff + j0 + u) * n_pc + pc) * 26;
      for (int t = 0; t < NV; t++) o[t] = tot[t];
    } else if (threadIdx.x == 0) {
      double* qa = qacc + (size_t)(fr.qoff + j0 + u) * QA_STRIDE;
      if (BWD != 1) {
        atomicAdd(&qa[QA_PHI_LR], tot[0]);
        for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_DPHI_LR + t], tot[1 + t]);
        for (int t = 0; t < 6; t++) atomicAdd(&qa[QA_H_LR + t], tot[4 + t]);
      }
      if (BWD != 0) {
        for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_G_QMMM_LR + t], tot[OB + t]);
        if (qmqm) {
          for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_G_QQ_LR + t], tot[OB + 3 + t]);
          atomicAdd(&qa[QA_DQ_QQ_LR], tot[OB + 6]);
          for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_DMU_QQ_LR + t], tot[OB + 7 + t]);
          for (int t = 0; t < 6; t++) atomicAdd(&qa[QA_DTH_QQ_LR + t], tot[OB + 10 + t]);
        }
      }
    }
  }
}

template <int BWD, int S>
__global__ __launch_bounds__(256) void k_project_qm(Grid g, FrameArg fa, int n_pc, const double2* __restrict__ smm,
                                                    size_t smm_stride, const double* __restrict__ Q,
                                                    const double* __restrict__ mu, const double* __restrict__ theta,
                                                    const double* __restrict__ qeff,
                                                    const double2* __restrict__ qtab,
                                                    const double2* __restrict__ sabc,
                                                    const double* __restrict__ kw, int qmqm,
                                                    double* __restrict__ qacc, double* __restrict__ det) {
  __shared__ double red[project_lds_doubles<BWD>()];
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  project_qm_item<BWD, S>(g, fr, f, blockIdx.x, blockIdx.y, n_pc, smm, smm_stride, Q, mu, theta, qeff, qtab, sabc,
                          kw, qmqm, qacc, det, red);
}

hipError_t launch_project_qm(const Grid& g, const FrameArg& fa, int max_nq, int total_nq, const double2* smm,
                             size_t smm_frame_stride, const double* Q, const double* mu, const double* theta,
                             int backward, int qmqm, Work& w, hipStream_t s) {
  if (max_nq == 0) return hipSuccess;
  // two sites per block (the per-k loads serve both); about 640 blocks in all:
  // enough k items per thread to amortise the block reduction
  constexpr int S = 2;
  const int site_blocks = (total_nq + S - 1) / S;
  int n_pc = (640 + site_blocks - 1) / (site_blocks > 0 ? site_blocks : 1);
  const int kblocks = (g.NCOL * (g.mz + 1) + 255) / 256;
  if (n_pc > kblocks) n_pc = kblocks;
  if (w.det_proj && n_pc > kDetPc) n_pc = kDetPc;
  if (n_pc < 1) n_pc = 1;
  dim3 grid((max_nq + S - 1) / S, n_pc, fa.n_frames);
#define PQ(B)                                                                                                  \
  hipLaunchKernelGGL((k_project_qm<B, S>), grid, dim3(256), 0, s, g, fa, n_pc, smm, smm_frame_stride, Q, mu, \
                     theta, w.qeff, w.qm_tab, w.sabc, w.kw, qmqm, w.qacc, w.det_proj)
  if (backward == 2)
    PQ(2);
  else if (backward)
    PQ(1);
  else
    PQ(0);
#undef PQ
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !w.det_proj) return e;
  // partial t of the forward sums goes to slot QA_PHI_LR + t, of the adjoint sums to QA_G_QMMM_LR + t
  DetMap m{};
  if (backward != 1) m = det_range(m, QA_PHI_LR, 10);
  if (backward) m = det_range(m, QA_G_QMMM_LR, 16);
  return launch_det_reduce(fa, 1, max_nq, w.det_proj, n_pc, 26, m, w.qacc, QA_STRIDE, s);
}

// ------------------------------------------------------------------ MM gradients (backward hot loop)
// For MM atom i: V(R) = sum_k W(k) e^{-i k.R}, W = (8 pi/V) g S'_QM, gives
// dL/dq_i = Re V(R_i) and dL/dR_i = q_i grad Re V(R_i).  Lanes own atoms
// (A per lane for instruction-level parallelism).  For each column (nx,ny)
// the nz sum is one Horner chain in u = e^{-i kz0 z} over n' = nz + mz =
// 0..2mz, together with its derivative for the nz-weighted sum of the z
// gradient: eight FMAs per k, the weights W being wave-uniform scalar loads.
// The column factor c = e^{-i(kx x + ky y)} e^{i mz kz0 z} follows the
// columns by complex recurrences in ny and nx, so no per-atom table is read.
template <int MZ>
DEV void horner_column(const double2* __restrict__ wc, int mz, double2 u, double& pr, double& pi, double& dr,
                       double& di) {
  const int top = MZ > 0 ? 2 * MZ : 2 * mz;
  pr = wc[top].x;
  pi = wc[top].y;
  dr = 0.0;
  di = 0.0;
  if (MZ > 0) {
#pragma unroll
    for (int n = 2 * MZ - 1; n >= 0; n--) {
      const double2 w = wc[n];
      const double tr = fma(dr, u.x, fma(-di, u.y, pr));
      di = fma(dr, u.y, fma(di, u.x, pi));
      dr = tr;
      const double t2 = fma(pr, u.x, fma(-pi, u.y, w.x));
      pi = fma(pr, u.y, fma(pi, u.x, w.y));
      pr = t2;
    }
  } else {
#pragma unroll 4
    for (int n = top - 1; n >= 0; n--) {
      const double2 w = wc[n];
      const double tr = fma(dr, u.x, fma(-di, u.y, pr));
      di = fma(dr, u.y, fma(di, u.x, pi));
      dr = tr;
      const double t2 = fma(pr, u.x, fma(-pi, u.y, w.x));
      pi = fma(pr, u.y, fma(pi, u.x, w.y));
      pr = t2;
    }
  }
}

template <int MZ, int A>
__global__ __launch_bounds__(256) void k_force_mm(Grid g, FrameArg fa, int kc_n, const double* __restrict__ mm4,
                                                  int cap_mm, const double2* __restrict__ wk,
                                                  double* __restrict__ fpart) {
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  const int i0 = blockIdx.x * 256 * A;
  if (i0 >= fr.nm) return;
  const int kc = blockIdx.y;
  const int per = (g.NCOL + kc_n - 1) / kc_n;
  const int c0 = kc * per, c1 = min(g.NCOL, c0 + per);
  const int mz = MZ > 0 ? MZ : g.mz;
  double2 u[A], c[A], crow[A], wy[A], wx[A];
  double aphi[A], agx[A], agy[A], agz[A];
  const int nx0 = c0 / g.NY, iy0 = c0 - nx0 * g.NY;
#pragma unroll
  for (int a = 0; a < A; a++) {
    const int i = min(i0 + threadIdx.x + 256 * a, fr.nm - 1);
    const int row = fr.moff + i;
    const double x = mm4[row] * fr.inv_box[0];
    const double y = mm4[(size_t)cap_mm + row] * fr.inv_box[1];
    const double z = mm4[(size_t)2 * cap_mm + row] * fr.inv_box[2];
    double s, co;
    sincospi(2.0 * z, &s, &co);
    u[a] = make_double2(co, -s);
    sincospi(2.0 * y, &s, &co);
    wy[a] = make_double2(co, -s);
    sincospi(2.0 * x, &s, &co);
    wx[a] = make_double2(co, -s);
    // row start (nx0, ny=-my) and column start (nx0, ny0), both times e^{+i mz kz0 z}
    sincospi(2.0 * ((double)mz * z - (double)nx0 * x + (double)g.my * y), &s, &co);
    crow[a] = make_double2(co, s);
    sincospi(2.0 * ((double)mz * z - (double)nx0 * x - (double)(iy0 - g.my) * y), &s, &co);
    c[a] = make_double2(co, s);
    aphi[a] = agx[a] = agy[a] = agz[a] = 0.0;
  }
  const double2* __restrict__ wf = wk + (size_t)f * g.KF;
  int nx = nx0, iy = iy0;
  for (int col = c0; col < c1; col++) {
    if (col != c0) {
      if (iy == g.NY) {  // next row
        iy = 0;
        nx++;
#pragma unroll
        for (int a = 0; a < A; a++) {
          crow[a] = cmul(crow[a], wx[a]);
          c[a] = crow[a];
        }
      } else {
#pragma unroll
        for (int a = 0; a < A; a++) c[a] = cmul(c[a], wy[a]);
      }
    }
    const double2* __restrict__ wc = wf + (size_t)col * g.NZ;
    double pr[A], pi[A], dr[A], di[A];
    if (A == 1) {
      horner_column<MZ>(wc, mz, u[0], pr[0], pi[0], dr[0], di[0]);
    } else {
      // two atoms share every scalar load of W
      const int top = 2 * mz;
#pragma unroll
      for (int a = 0; a < A; a++) {
        pr[a] = wc[top].x;
        pi[a] = wc[top].y;
        dr[a] = di[a] = 0.0;
      }
#pragma unroll 8
      for (int n = top - 1; n >= 0; n--) {
        const double2 w = wc[n];
#pragma unroll
        for (int a = 0; a < A; a++) {
          const double tr = fma(dr[a], u[a].x, fma(-di[a], u[a].y, pr[a]));
          di[a] = fma(dr[a], u[a].y, fma(di[a], u[a].x, pi[a]));
          dr[a] = tr;
          const double t2 = fma(pr[a], u[a].x, fma(-pi[a], u[a].y, w.x));
          pi[a] = fma(pr[a], u[a].y, fma(pi[a], u[a].x, w.y));
          pr[a] = t2;
        }
      }
    }
    const double fny = (double)(iy - g.my), fnx = (double)nx;
#pragma unroll
    for (int a = 0; a < A; a++) {
      // V_col = c P~,  sum_n n W_n u^n (times the folded phase) = u D~ - mz P~
      const double2 cP = cmul(c[a], make_double2(pr[a], pi[a]));
      const double2 uD = cmul(u[a], make_double2(dr[a], di[a]));
      const double zr = uD.x - mz * pr[a], zi = uD.y - mz * pi[a];
      const double imz = c[a].x * zi + c[a].y * zr;
      aphi[a] += cP.x;
      agx[a] += fnx * cP.y;
      agy[a] += fny * cP.y;
      agz[a] += imz;
    }
    iy++;
  }
  const double kx0 = 2.0 * kPi * fr.inv_box[0], ky0 = 2.0 * kPi * fr.inv_box[1], kz0 = 2.0 * kPi * fr.inv_box[2];
#pragma unroll
  for (int a = 0; a < A; a++) {
    const int i = i0 + threadIdx.x + 256 * a;
    if (i < fr.nm) {
      double* o = fpart + ((size_t)kc * cap_mm + fr.moff + i) * 4;
      o[0] = aphi[a];
      o[1] = kx0 * agx[a];
      o[2] = ky0 * agy[a];
      o[3] = kz0 * agz[a];
    }
  }
}

// Matrix-core form of the same sums.  For a tile of 16 atoms and 16 columns
//   P[a][c]  = sum_nz E[a][nz] W[nz][c],   Pz[a][c] = sum_nz E[a][nz] nz W[nz][c],
//   E[a][nz] = e^{-i nz kz0 z_a},
// are complex products with the contraction over nz, four nz per
// ------------------------------------------------------------------ matrix-core adjoint
// For MM atom i and column c, with the folded weights of k_sfac_qm:
//   P(i,c)  = W(c,0) + sum_p [Ap cos(p kz0 z_i) - i Am sin(p kz0 z_i)]
//   Pz(i,c) = sum_p p [Am cos(p kz0 z_i) - i Ap sin(p kz0 z_i)]
// Re P, Im P, Re Pz, Im Pz are four real contractions of the z table
// (atoms x K, A operand, held in registers for the whole wave) with the
// folded weights (K x columns, B operand, fragment order).  The epilogue
// multiplies by c = e^{-i(kx x + ky y)} from the phase tables and accumulates
// per atom: Re(cP) (potential), nx Im(cP), ny Im(cP) and Im(c Pz) (forces
// up to the factors kx0, ky0, kz0).  AT tiles of 16 atoms per wave share the
// B operand.  The four waves of a block (different atoms, same columns) read
// each column group's B operand from LDS: the block copies it there once,
// double buffered, the next group's copy in flight during the contraction.
template <int NK, int AT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AT == 1 ? 3 : 1))) void k_force_mm_mfma(Grid g, FrameArg fa, int kc_n, int cap_mm,
                                                       const double2* __restrict__ tab,
                                                       const double* __restrict__ ztab,
                                                       const double* __restrict__ wfrag,
                                                       const double2* __restrict__ wk0, double* __restrict__ fpart) {
  __shared__ __align__(16) double bsh[2][NK * 256];
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int(threadIdx.x >> 6);
  if (blockIdx.x * 64 * AT >= fr.nm) return;  // uniform over the block
  // waves past the last atom still take part in the staging (their atoms are clamped, nothing is written)
  const int a0 = (blockIdx.x * 4 + wave) * 16 * AT;
  const int kc = blockIdx.y;
  const int per = (g.NG + kc_n - 1) / kc_n;
  const int gbeg = kc * per, gend = min(g.NG, gbeg + per);
  const int li = lane & 15, lk = lane >> 4;
  // A operands of every K step: z table of atom a0 + 16t + li, entry 4s + lk
  double za[AT][NK];
#pragma unroll
  for (int t = 0; t < AT; t++) {
    const int aA = min(a0 + 16 * t + li, fr.nm - 1);
    const double* __restrict__ zr = ztab + (size_t)(fr.moff + aA) * g.ZKP + lk;
#pragma unroll
    for (int st = 0; st < NK; st++) za[t][st] = zr[4 * st];
  }
  double acc0[AT][4], acc1[AT][4], acc2[AT][4], acc3[AT][4];
  int arow[AT][4];
#pragma unroll
  for (int t = 0; t < AT; t++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      acc0[t][r] = acc1[t][r] = acc2[t][r] = acc3[t][r] = 0.0;
      arow[t][r] = fr.moff + min(a0 + 16 * t + lk + 4 * r, fr.nm - 1);
    }
  const double* __restrict__ wfr = wfrag + (size_t)f * g.NG * NK * 256 + threadIdx.x;
  double stg[NK];
  if (gbeg < gend) {
#pragma unroll
    for (int u = 0; u < NK; u++) stg[u] = wfr[(size_t)gbeg * NK * 256 + 256 * u];
#pragma unroll
    for (int u = 0; u < NK; u++) bsh[0][threadIdx.x + 256 * u] = stg[u];
  }
  __syncthreads();
  int cur = 0;
  for (int grp = gbeg; grp < gend; grp++) {
    const bool more = grp + 1 < gend;
    if (more) {
#pragma unroll
      for (int u = 0; u < NK; u++) stg[u] = wfr[(size_t)(grp + 1) * NK * 256 + 256 * u];
    }
    const int col = grp * 16 + li;
    const bool cok = col < g.NCOL;
    const int colc = cok ? col : g.NCOL - 1;
    const int nx = colc / g.NY, iy = colc - nx * g.NY;
    // column phases of the epilogue, loaded ahead of the contraction
    double2 ex[AT][4], ey[AT][4];
#pragma unroll
    for (int t = 0; t < AT; t++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const double2* __restrict__ row = tab + (size_t)arow[t][r] * g.NXY;
        ex[t][r] = row[nx];
        ey[t][r] = row[g.NX + iy];
      }
    const double2 w0 = wk0[(size_t)f * g.NG * 16 + grp * 16 + li];
    const double* __restrict__ wg = bsh[cur] + 2 * lane;  // B values of a K step: 2 lane + {0, 1, 128, 129}
    v4d Pr[AT], Pi[AT], Zr[AT], Zi[AT];
#pragma unroll
    for (int t = 0; t < AT; t++) {
      Pr[t] = v4d{w0.x, w0.x, w0.x, w0.x};
      Pi[t] = v4d{w0.y, w0.y, w0.y, w0.y};
      Zr[t] = v4d{0.0, 0.0, 0.0, 0.0};
      Zi[t] = v4d{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int st = 0; st < NK; st++) {
      const double2 u = *reinterpret_cast<const double2*>(wg + st * 256);
      const double2 v = *reinterpret_cast<const double2*>(wg + st * 256 + 128);
      const double b0 = u.x, b1 = u.y, b2 = v.x, b3 = v.y;
#pragma unroll
      for (int t = 0; t < AT; t++) {
        Pr[t] = mfma4(za[t][st], b0, Pr[t]);
        Pi[t] = mfma4(za[t][st], b1, Pi[t]);
        Zr[t] = mfma4(za[t][st], b2, Zr[t]);
        Zi[t] = mfma4(za[t][st], b3, Zi[t]);
      }
    }
    const double fnx = (double)nx, fny = (double)(iy - g.my);
    if (cok) {
#pragma unroll
      for (int t = 0; t < AT; t++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          // c = e^{-i(kx x + ky y)} = conj(e^{i kx x} e^{i ky y})
          const double2 c = cconj(cmul(ex[t][r], ey[t][r]));
          const double cpr = c.x * Pr[t][r] - c.y * Pi[t][r];
          const double cpi = c.x * Pi[t][r] + c.y * Pr[t][r];
          const double czi = c.x * Zi[t][r] + c.y * Zr[t][r];
          acc0[t][r] += cpr;
          acc1[t][r] += fnx * cpi;
          acc2[t][r] += fny * cpi;
          acc3[t][r] += czi;
        }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < NK; u++) bsh[cur ^ 1][threadIdx.x + 256 * u] = stg[u];
    }
    __syncthreads();
    cur ^= 1;
  }
  // sum over the 16 columns held by lanes with the same lk
#pragma unroll
  for (int t = 0; t < AT; t++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        acc0[t][r] += __shfl_xor(acc0[t][r], o, 64);
        acc1[t][r] += __shfl_xor(acc1[t][r], o, 64);
        acc2[t][r] += __shfl_xor(acc2[t][r], o, 64);
        acc3[t][r] += __shfl_xor(acc3[t][r], o, 64);
      }
    }
  if (li == 0) {
    const double kx0 = 2.0 * kPi * fr.inv_box[0], ky0 = 2.0 * kPi * fr.inv_box[1], kz0 = 2.0 * kPi * fr.inv_box[2];
#pragma unroll
    for (int t = 0; t < AT; t++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int a = a0 + 16 * t + lk + 4 * r;
        if (a < fr.nm) {
          double* o = fpart + ((size_t)kc * cap_mm + fr.moff + a) * 4;
          o[0] = acc0[t][r];
          o[1] = kx0 * acc1[t][r];
          o[2] = ky0 * acc2[t][r];
          o[3] = kz0 * acc3[t][r];
        }
      }
  }
}

// Matrix-core adjoint with the y phases of the block's atoms staged in LDS
// once: the epilogue reads e^{i ky y} for every (atom, column) of every
// column group, and from LDS these re-reads no longer compete for L2 with the
// other blocks (from L2 they spilled to HBM).  The B operand (the folded
// weights of one frame, ~2 MB at |n| <= 24) is read from L2.  The LDS tile is
// NY rows of (16 WV + 1) complex entries, ny-major (one pad entry per row
// spreads the 16 columns a wave reads at once over all banks), dynamic:
// WV = 4 waves (64 atoms) per block, or 2 (32 atoms) when the 64-atom tile
// of a large y grid does not fit 64 KB.
// On gfx950 an FP64 matrix-core instruction and a VALU instruction of the
// same SIMD do not execute together, so every VALU instruction of the column
// loop lengthens it.  The loop therefore does no address arithmetic per load:
// B and the x phases are buffer loads from a wave-uniform resource with one
// per-lane offset and uniform (scalar) offsets per K step or atom row; the
// column (nx, ny) of a lane advances without a division; a group's x phases
// are loaded at its start and used in its epilogue, after the contraction;
// the nz = 0 weight is added in the epilogue rather than copied into the
// accumulators; the epilogue is fused multiply-adds with no branch (padded
// columns have zero weights).  The B fragments of the next BD K steps are in
// flight through a register ring that runs across groups, its order pinned
// with scheduling barriers (left alone, the compiler drained each step's
// loads before the next).  Buffer loads past the end of their resource
// return zero, so the atom rows of a partial tile need no clamping (their
// results are not stored).
// The grid is one-dimensional per frame, atom-tile major: the kc_n blocks of
// one atom tile are consecutive logical blocks.  With xcd_remap (single
// frame) consecutive logical blocks are placed on one XCD, so that the blocks
// sharing an atom tile read its phase rows through one L2.

// One adjoint work item: atom tile `tile` (16 WV atoms) and column chunk kc of
// kc_n of frame f, all 64 WV threads of the block; eysh holds
// eyl_lds_bytes(g, WV), or with HY (half y) eyl_half_lds_bytes(g): only the
// rows ny >= 0, a column with ny < 0 taking the conjugate of row -ny.
// Returns (uniformly) for a tile past the frame's atoms; waves past the last
// atom return after the staging barrier (no barrier follows it).
template <int NK, int WV, bool HY>
DEV void force_mm_eyl_item(const Grid& g, const FrameDev& fr, int f, int tile, int kc, int kc_n, int cap_mm,
                           const double2* __restrict__ tab, const double* __restrict__ ztab,
                           const double* __restrict__ wfrag, const double2* __restrict__ wk0,
                           double* __restrict__ fpart, double2* eysh) {
  constexpr int NA = 16 * WV;  // atoms per block
  constexpr int ES = NA + 1;   // LDS row stride in entries
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int(threadIdx.x >> 6);
  const int ablk = tile * NA;
  if (ablk >= fr.nm) return;  // uniform over the block
  {
    // entry e = a NY + c of the tile; (a, c) advance by the block size
    // without a division per entry (VALU instructions here delay the
    // matrix-core issue of the other waves on the SIMD)
    constexpr int NT = 64 * WV;
    const int rows = HY ? g.my + 1 : g.NY;  // LDS row c holds iy = c (HY: iy = my + c, ny = c)
    const int da = NT / rows, dc = NT - da * rows;
    int a = threadIdx.x / rows, c = threadIdx.x - a * rows;
    const double2* __restrict__ src = tab + (size_t)fr.moff * g.NXY + g.NX + (HY ? g.my : 0);
    for (int e = threadIdx.x; e < NA * rows; e += NT) {
      eysh[c * ES + a] = src[(size_t)min(ablk + a, fr.nm - 1) * g.NXY + c];
      a += da;
      c += dc;
      if (c >= rows) {
        c -= rows;
        a++;
      }
    }
  }
  __syncthreads();
  const int a0 = ablk + wave * 16;
  if (a0 >= fr.nm) return;  // no barrier after this point
  const int per = (g.NG + kc_n - 1) / kc_n;
  const int gbeg = kc * per, gend = min(g.NG, gbeg + per);
  const int li = lane & 15, lk = lane >> 4;
  double za[NK];
  {
    const int aA = min(a0 + li, fr.nm - 1);
    const double* __restrict__ zr = ztab + (size_t)(fr.moff + aA) * g.ZKP + lk;
#pragma unroll
    for (int st = 0; st < NK; st++) za[st] = zr[4 * st];
  }
  double acc0[4], acc1[4], acc2[4], acc3[4];
#pragma unroll
  for (int r = 0; r < 4; r++) acc0[r] = acc1[r] = acc2[r] = acc3[r] = 0.0;
  // x phases of this frame's atoms (the launcher keeps one frame's table
  // below 2 GB): row a0 + lk at byte xoff, rows 4 apart at a uniform stride
  const __amdgpu_buffer_rsrc_t xr = buf_rsrc(tab + (size_t)fr.moff * g.NXY, (unsigned)fr.nm * g.NXY * 16u);
  const int xoff = (a0 + lk) * g.NXY * 16;
  const int xrow = 4 * g.NXY * 16;
  const int erow = wave * 16 + lk;  // LDS entry of row r = 0; rows r are 4 entries apart
  const int q16 = 16 / g.NY, r16 = 16 - q16 * g.NY;
  auto load_ex = [&](int nx, double2 (&ex)[4]) {
    const int vo = xoff + min(nx, g.NX - 1) * 16;
#pragma unroll
    for (int r = 0; r < 4; r++) ex[r] = buf_load_c64(xr, vo, r * xrow);
  };
  const double2* __restrict__ w0f = wk0 + (size_t)f * g.NG * 16;
  const double* __restrict__ wff = wfrag + (size_t)f * g.NG * NK * 256;
  // B operand ring: the fragments of K step st + BD are in flight while step
  // st is contracted, across the end of a group into the next one (BD divides
  // NK, so a K step has the same ring slot in every group)
  constexpr int BD = NK % 3 == 0 ? 3 : (NK % 4 == 0 && NK <= 4) ? 4 : 2;
  static_assert(NK % BD == 0, "ring depth must divide the K steps");
  double bq[BD][4];
  auto wrsrc = [&](int grp) { return buf_rsrc(wff + (size_t)grp * NK * 256, NK * 256 * 8); };
  // a lane's B values of K step st: matrices 0, 1 and 2, 3 as two 16-byte loads
  auto load_b = [&](__amdgpu_buffer_rsrc_t wr, int st, double (&b)[4]) {
    const double2 u = buf_load_c64(wr, lane * 16, st * 2048);
    const double2 v = buf_load_c64(wr, lane * 16, st * 2048 + 1024);
    b[0] = u.x;
    b[1] = u.y;
    b[2] = v.x;
    b[3] = v.y;
  };
  int col = gbeg * 16 + li;
  int nx = col / g.NY, iy = col - nx * g.NY;
  {
    const __amdgpu_buffer_rsrc_t w = wrsrc(min(gbeg, g.NG - 1));  // an empty chunk loads and discards
#pragma unroll
    for (int st = 0; st < BD; st++) load_b(w, st, bq[st]);
  }
  for (int grp = gbeg; grp < gend; grp++) {
    // the x phases of this group arrive while it is contracted
    double2 ex[4];
    load_ex(nx, ex);
    // the next group this wave contracts (the last one repeats itself)
    const __amdgpu_buffer_rsrc_t wn = wrsrc(min(grp + 1, gend - 1));
    const __amdgpu_buffer_rsrc_t wr = wrsrc(grp);
    const double2 w0 = w0f[grp * 16 + li];
    v4d Pr = v4d{0.0, 0.0, 0.0, 0.0}, Pi = Pr, Zr = Pr, Zi = Pr;
    // the order is fixed as written (the compiler would otherwise trade the
    // loads in flight for registers): per K step four independent
    // matrix-core chains, then the loads of step st + BD into the freed slot
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < NK; st++) {
      double (&b)[4] = bq[st % BD];
      Pr = mfma4(za[st], b[0], Pr);
      Pi = mfma4(za[st], b[1], Pi);
      Zr = mfma4(za[st], b[2], Zr);
      Zi = mfma4(za[st], b[3], Zi);
      if (st + BD < NK)
        load_b(wr, st + BD, b);
      else
        load_b(wn, st + BD - NK, b);
      __builtin_amdgcn_sched_barrier(0);
    }
    // columns past NCOL (in the last group) have zero weights: their terms
    // vanish without a branch
    const double fnx = (double)nx, fny = (double)(iy - g.my);
    // HY: row |ny|, conjugated for ny < 0
    const int yrow = HY ? (iy < g.my ? g.my - iy : iy - g.my) : iy;
    const double sy = (HY && iy < g.my) ? -1.0 : 1.0;
    const double2* __restrict__ ey = eysh + yrow * ES + erow;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      // c = e^{-i(kx x + ky y)} = conj(e^{i kx x} e^{i ky y}) = cr - i s
      double2 e = ey[4 * r];
      if (HY) e.y *= sy;
      const double pr = Pr[r] + w0.x, pi = Pi[r] + w0.y;
      const double cr = fma(ex[r].x, e.x, -ex[r].y * e.y);
      const double s = fma(ex[r].x, e.y, ex[r].y * e.x);
      const double cpi = fma(cr, pi, -s * pr);
      acc0[r] = fma(cr, pr, acc0[r]);
      acc0[r] = fma(s, pi, acc0[r]);
      acc1[r] = fma(fnx, cpi, acc1[r]);
      acc2[r] = fma(fny, cpi, acc2[r]);
      acc3[r] = fma(cr, Zi[r], acc3[r]);
      acc3[r] = fma(-s, Zr[r], acc3[r]);
    }
    // next column of this lane: 16 further, (nx, iy) without a division
    iy += r16;
    nx += q16;
    if (iy >= g.NY) {
      iy -= g.NY;
      nx++;
    }
  }
  // sum over the 16 columns held by lanes with the same lk
#pragma unroll
  for (int r = 0; r < 4; r++) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      acc0[r] += __shfl_xor(acc0[r], o, 64);
      acc1[r] += __shfl_xor(acc1[r], o, 64);
      acc2[r] += __shfl_xor(acc2[r], o, 64);
      acc3[r] += __shfl_xor(acc3[r], o, 64);
    }
  }
  if (li == 0) {
    const double kx0 = 2.0 * kPi * fr.inv_box[0], ky0 = 2.0 * kPi * fr.inv_box[1], kz0 = 2.0 * kPi * fr.inv_box[2];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int a = a0 + lk + 4 * r;
      if (a < fr.nm) {
        double* o = fpart + ((size_t)kc * cap_mm + fr.moff + a) * 4;
        o[0] = acc0[r];
        o[1] = kx0 * acc1[r];
        o[2] = ky0 * acc2[r];
        o[3] = kz0 * acc3[r];
      }
    }
  }
}

template <int NK, int WV, bool HY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_force_mm_eyl(
    Grid g, FrameArg fa, int kc_n, int xcd_remap, int cap_mm, const double2* __restrict__ tab,
    const double* __restrict__ ztab, const double* __restrict__ wfrag, const double2* __restrict__ wk0,
    double* __restrict__ fpart) {
  extern __shared__ double2 eysh[];  // [NY][16 WV + 1]
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  int bid = blockIdx.x;
  if (xcd_remap) {
    const int per = (int)gridDim.x / 8;
    if (bid < 8 * per) bid = (bid % 8) * per + bid / 8;
  }
  const int tile = bid / kc_n, kc = bid - tile * kc_n;
  force_mm_eyl_item<NK, WV, HY>(g, fr, f, tile, kc, kc_n, cap_mm, tab, ztab, wfrag, wk0, fpart, eysh);
}

// Warp-specialised matrix-core adjoint: in a block of eight waves, waves 0-3
// (one 16-atom tile each) only issue the contraction (B operand from L2,
// where the folded weights stay resident) and write their four accumulator
// tiles to LDS; waves 4-7 apply the epilogue of the previous column group
// (phase tables, complex products, per-atom sums), so that no FP64 VALU work
// sits between the matrix-core instructions of a wave.  One barrier per
// column group; the tile exchange is double buffered (64 KB, two blocks per CU).
template <int NK>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_force_mm_ws(
    Grid g, FrameArg fa, int kc_n, int cap_mm, const double2* __restrict__ tab, const double* __restrict__ ztab,
    const double* __restrict__ wfrag, const double2* __restrict__ wk0, double* __restrict__ fpart) {
  __shared__ double psh[2][4][16][64];
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uniform_int(tid >> 6);
  const bool mma = wave < 4;
  const int wt = wave & 3;
  if (blockIdx.x * 64 >= fr.nm) return;  // uniform over the block
  const int a0 = (blockIdx.x * 4 + wt) * 16;
  const int kc = blockIdx.y;
  const int per = (g.NG + kc_n - 1) / kc_n;
  // an empty column range (more chunks than groups) still writes its zero partial sums
  const int gbeg = kc * per, gend = min(g.NG, gbeg + per);
  const int li = lane & 15, lk = lane >> 4;
  // matrix-core waves: A operands of every K step
  double za[NK];
  if (mma) {
    const int aA = min(a0 + li, fr.nm - 1);
    const double* __restrict__ zr = ztab + (size_t)(fr.moff + aA) * g.ZKP + lk;
#pragma unroll
    for (int st = 0; st < NK; st++) za[st] = zr[4 * st];
  }
  // epilogue waves: per-atom sums
  double acc0[4], acc1[4], acc2[4], acc3[4];
  int arow[4];
#pragma unroll
  for (int r = 0; r < 4; r++) {
    acc0[r] = acc1[r] = acc2[r] = acc3[r] = 0.0;
    arow[r] = fr.moff + min(a0 + lk + 4 * r, fr.nm - 1);
  }
  for (int it = gbeg; it <= gend && gbeg < gend; it++) {
    const int cur = (it - gbeg) & 1;
    if (mma) {
      if (it < gend) {
        const double2 w0 = wk0[(size_t)f * g.NG * 16 + it * 16 + li];
        v4d Pr = v4d{w0.x, w0.x, w0.x, w0.x}, Pi = v4d{w0.y, w0.y, w0.y, w0.y};
        v4d Zr = v4d{0.0, 0.0, 0.0, 0.0}, Zi = v4d{0.0, 0.0, 0.0, 0.0};
        const double* __restrict__ wg = wfrag + ((size_t)f * g.NG + it) * NK * 256 + 2 * lane;
#pragma unroll
        for (int st = 0; st < NK; st++) {
          const double2 u = *reinterpret_cast<const double2*>(wg + st * 256);
          const double2 v = *reinterpret_cast<const double2*>(wg + st * 256 + 128);
          const double b0 = u.x, b1 = u.y, b2 = v.x, b3 = v.y;
          Pr = mfma4(za[st], b0, Pr);
          Pi = mfma4(za[st], b1, Pi);
          Zr = mfma4(za[st], b2, Zr);
          Zi = mfma4(za[st], b3, Zi);
        }
        double* __restrict__ pt = &psh[cur][wt][0][lane];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          pt[(0 + r) * 64] = Pr[r];
          pt[(4 + r) * 64] = Pi[r];
          pt[(8 + r) * 64] = Zr[r];
          pt[(12 + r) * 64] = Zi[r];
        }
      }
    } else if (it > gbeg) {
      const int grp = it - 1;
      const int col = grp * 16 + li;
      if (col < g.NCOL) {
        const int nx = col / g.NY, iy = col - nx * g.NY;
        const double fnx = (double)nx, fny = (double)(iy - g.my);
        const double* __restrict__ pt = &psh[cur ^ 1][wt][0][lane];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const double2* __restrict__ row = tab + (size_t)arow[r] * g.NXY;
          const double2 c = cconj(cmul(row[nx], row[g.NX + iy]));
          const double pr = pt[(0 + r) * 64], pi = pt[(4 + r) * 64];
          const double zr = pt[(8 + r) * 64], zi = pt[(12 + r) * 64];
          const double cpi = c.x * pi + c.y * pr;
          acc0[r] += c.x * pr - c.y * pi;
          acc1[r] += fnx * cpi;
          acc2[r] += fny * cpi;
          acc3[r] += c.x * zi + c.y * zr;
        }
      }
    }
    __syncthreads();
  }
  if (mma) return;
  // sum over the 16 columns held by lanes with the same lk
#pragma unroll
  for (int r = 0; r < 4; r++) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      acc0[r] += __shfl_xor(acc0[r], o, 64);
      acc1[r] += __shfl_xor(acc1[r], o, 64);
      acc2[r] += __shfl_xor(acc2[r], o, 64);
      acc3[r] += __shfl_xor(acc3[r], o, 64);
    }
  }
  if (li == 0) {
    const double kx0 = 2.0 * kPi * fr.inv_box[0], ky0 = 2.0 * kPi * fr.inv_box[1], kz0 = 2.0 * kPi * fr.inv_box[2];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int a = a0 + lk + 4 * r;
      if (a < fr.nm) {
        double* o = fpart + ((size_t)kc * cap_mm + fr.moff + a) * 4;
        o[0] = acc0[r];
        o[1] = kx0 * acc1[r];
        o[2] = ky0 * acc2[r];
        o[3] = kz0 * acc3[r];
      }
    }
  }
}

template <int MZ, int A>
static void launch_force_mm_t(dim3 grid, hipStream_t s, const Grid& g, const FrameArg& fa, int kc, int cap_mm,
                              Work& w) {
  hipLaunchKernelGGL((k_force_mm<MZ, A>), grid, dim3(256), 0, s, g, fa, kc, w.mm4, cap_mm, w.wk, w.fpart);
}

hipError_t launch_force_mm(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                           hipStream_t s) {
  if (max_nm == 0) return hipSuccess;
  if (t.fp32r) return launch_force_mm32(g, t, fa, max_nm, cap_mm, w, s);
  if (t.bwd_ilp == 6 && mfma_bwd_eyl_ok(g)) {  // y phases in LDS: 64 (or 32) atoms per block
    if (!tab32_ok(g, max_nm)) return hipErrorInvalidValue;  // the API rejects such frames first
    const bool hy = eyl_half_y(g);
    const int wv = hy ? 4 : eyl_waves(g);
    dim3 grid(((max_nm + 16 * wv - 1) / (16 * wv)) * t.kc, 1, fa.n_frames);
    const size_t lds = hy ? eyl_half_lds_bytes(g) : eyl_lds_bytes(g, wv);
    const int xcd = (t.bwd_xcd && fa.n_frames == 1) ? 1 : 0;
#define FE(N)                                                                                                       \
  case N:                                                                                                           \
    if (hy)                                                                                                         \
      hipLaunchKernelGGL((k_force_mm_eyl<N, 4, true>), grid, dim3(256), lds, s, g, fa, t.kc, xcd, cap_mm, w.mm_xy, \
                         w.mm_ztab, w.wfrag, w.wk0, w.fpart);                                                       \
    else if (wv == 4)                                                                                               \
      hipLaunchKernelGGL((k_force_mm_eyl<N, 4, false>), grid, dim3(256), lds, s, g, fa, t.kc, xcd, cap_mm,         \
                         w.mm_xy, w.mm_ztab, w.wfrag, w.wk0, w.fpart);                                              \
    else                                                                                                            \
      hipLaunchKernelGGL((k_force_mm_eyl<N, 2, false>), grid, dim3(128), lds, s, g, fa, t.kc, xcd, cap_mm,         \
                         w.mm_xy, w.mm_ztab, w.wfrag, w.wk0, w.fpart);                                              \
    break;
    switch (g.NK2) { FE(2) FE(4) FE(6) FE(8) FE(10) FE(12) FE(14) FE(16) default: return hipErrorInvalidValue; }
#undef FE
    return hipGetLastError();
  }
  if (t.bwd_ilp == 5 && mfma_bwd_ok(g)) {  // warp-specialised matrix-core path: 64 atoms per 512-thread block
    dim3 grid((max_nm + 63) / 64, t.kc, fa.n_frames);
#define FW(N)                                                                                                 \
  case N:                                                                                                     \
    hipLaunchKernelGGL((k_force_mm_ws<N>), grid, dim3(512), 0, s, g, fa, t.kc, cap_mm, w.mm_xy, w.mm_ztab, \
                       w.wfrag, w.wk0, w.fpart);                                                              \
    break;
    switch (g.NK2) { FW(2) FW(4) FW(6) FW(8) FW(10) FW(12) FW(14) FW(16) default: return hipErrorInvalidValue; }
#undef FW
    return hipGetLastError();
  }
  if (t.bwd_ilp >= 3 && mfma_bwd_ok(g)) {  // matrix-core path: 64 (AT=1) or 128 (AT=2) atoms per block
    const int at = t.bwd_ilp == 4 ? 2 : 1;
    dim3 grid((max_nm + 64 * at - 1) / (64 * at), t.kc, fa.n_frames);
#define FM(N, AT)                                                                                          \
  hipLaunchKernelGGL((k_force_mm_mfma<N, AT>), grid, dim3(256), 0, s, g, fa, t.kc, cap_mm, w.mm_xy, w.mm_ztab, \
                     w.wfrag, w.wk0, w.fpart)
#define FMC(N)              \
  case N:                   \
    if (at == 2)            \
      FM(N, 2);             \
    else                    \
      FM(N, 1);             \
    break;
    switch (g.NK2) { FMC(2) FMC(4) FMC(6) FMC(8) FMC(10) FMC(12) FMC(14) FMC(16) default: return hipErrorInvalidValue; }
#undef FMC
#undef FM
    return hipGetLastError();
  }
  const int A = t.bwd_ilp == 1 ? 1 : 2;
  dim3 grid((max_nm + 256 * A - 1) / (256 * A), t.kc, fa.n_frames);
  if (A == 2) {
    launch_force_mm_t<0, 2>(grid, s, g, fa, t.kc, cap_mm, w);
  } else {
    switch (g.mz) {
      case 8: launch_force_mm_t<8, 1>(grid, s, g, fa, t.kc, cap_mm, w); break;
      case 16: launch_force_mm_t<16, 1>(grid, s, g, fa, t.kc, cap_mm, w); break;
      case 20: launch_force_mm_t<20, 1>(grid, s, g, fa, t.kc, cap_mm, w); break;
      case 24: launch_force_mm_t<24, 1>(grid, s, g, fa, t.kc, cap_mm, w); break;
      case 32: launch_force_mm_t<32, 1>(grid, s, g, fa, t.kc, cap_mm, w); break;
      default: launch_force_mm_t<0, 1>(grid, s, g, fa, t.kc, cap_mm, w); break;
    }
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ real space
// Screened tensors of erfc(a r)/r about the QM site, r = R_qm - R_mm
// (SI, screened tensors with kappa = alpha):
//   psi0 = f1, psi1 = -r f3, psi2 = 1/2 (3 r r f5 - I f3),
//   psi3 = 1/2 [ (r delta)_sym f5 - 5 r r r f7 ]
// contracted analytically with the moments.
template <typename T>
struct Radial {
  T f1, f3, f5, f7;
};

// erfcx(x) = e^{x^2} erfc(x) for x >= 0 from its Chebyshev expansion in
// t = (x - 3)/(x + 3) (orders 0..22, written by gen_erfcx.py beside this
// file: relative error below 1.1e-15 for x in [0, 8], 5.5e-15 up to 40),
// summed with Clenshaw's recurrence.  With e^{-x^2}, which the radial
// functions need anyway, it gives erfc without a second exponential and
// without the range branches of a general erfc.
__constant__ double kErfcxCheb[23] = {
    +3.29862774753036769e-01, -4.53661520537802065e-01, +1.60398340821562957e-01,
    -4.49081211511228248e-02, +9.64142865069569747e-03, -1.44250807774439545e-03,
    +1.00994367353799156e-04, +1.20850245344553003e-05, -3.62542060275375560e-06,
    +7.18681074247641496e-08, +8.91423585989821744e-08, -7.42156662495960609e-09,
    -2.38933657026587794e-09, +3.06223553548992515e-10, +7.78894538815108849e-11,
    -1.09737458292455838e-11, -3.09152073119177339e-12, +3.52543388172342203e-13,
    +1.39904521797716168e-13, -8.24603747683880858e-15, -6.63996142698932149e-15,
    -7.97834882475261098e-17, +3.04724123760409854e-16};

DEV double erfcx_pos(double x) {
  const double t = (x - 3.0) / (x + 3.0), t2 = 2.0 * t;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int n = 22; n >= 1; n--) {
    const double b0 = fma(t2, b1, kErfcxCheb[n] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(t, b1, kErfcxCheb[0] - b2);
}

template <typename T>
DEV Radial<T> radial(T r2, T a) {
  const T r = sqrt(r2);
  const T ex = exp(-a * a * r2);
  const T inv2 = T(1) / r2;
  const T c = T(1.1283791670955126) * a;  // 2 a / sqrt(pi)
  Radial<T> o;
  if constexpr (std::is_same<T, double>::value)
    o.f1 = ex * erfcx_pos(a * r) * (r * inv2);  // erfc(a r) / r
  else
    o.f1 = erfc(a * r) / r;
  o.f3 = (o.f1 + c * ex) * inv2;
  o.f5 = (o.f3 + T(2.0 / 3.0) * a * a * c * ex) * inv2;
  o.f7 = (o.f5 + T(4.0 / 15.0) * a * a * a * a * c * ex) * inv2;
  return o;
}

DEV void min_image(double& dx, double& dy, double& dz, const FrameDev& fr) {
  dx -= fr.box[0] * rint(dx * fr.inv_box[0]);
  dy -= fr.box[1] * rint(dy * fr.inv_box[1]);
  dz -= fr.box[2] * rint(dz * fr.inv_box[2]);
}

// QM side of the QM-MM real-space sum.  Forward: phi, grad phi, 1/2 grad grad phi.
// Backward: dL/dR_qm with the effective moments.
// Pairs within the cutoff are few among the (site, atom, image) triples a
// block tests (a few percent at rc <= L/2), and a wave whose lanes test
// different atoms would evaluate erfc and exp for a pair whenever any of its
// lanes has one.  Each wave therefore appends its lanes' pairs, in lane order,
// to a FIFO of its own in LDS and evaluates them 64 at a time, one pair per
// lane (the order is fixed, so the sums are too).
static constexpr int kPairFifo = 128;  // entries per wave (< 64 pending + up to 64 appended)

template <typename T>
constexpr int pair_fifo_bytes() {
  return 4 * kPairFifo * (5 * (int)sizeof(T) + (int)sizeof(int));
}

// LDS between the lanes of one wave: stores complete before other lanes read
DEV void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Lattice images n along one axis that can put b + n L within rc (at most
// nimg either side): a pair needs |b + n L| < rc on every axis.  The range is
// widened by 1e-9 L against rounding (a candidate too many only fails the
// distance test; it also covers the product with 1/L in place of a
// division).  A NaN offset gives the full range (its distance tests then
// fail), an infinite one an empty range; both ends stay within
// [-nimg - 1, nimg + 1] before conversion.
DEV void image_range(double b, double L, double inv_L, double rc, int nimg, int& lo, int& hi) {
  const double n = (double)nimg, w = rc + 1e-9 * L;
  lo = (int)fmin(fmax(ceil((-w - b) * inv_L), -n), n + 1.0);
  hi = (int)fmax(fmin(floor((w - b) * inv_L), n), -n - 1.0);
}

// Effective moments of one QM site as stored in qeff: Q, mu, theta (xx xy xz
// yy yz zz).
template <typename T>
struct SiteMoments {
  T Q, m0, m1, m2, t0, t1, t2, t3, t4, t5;
};

template <typename T>
DEV SiteMoments<T> site_moments(const double* qe) {
  return SiteMoments<T>{(T)qe[0], (T)qe[1], (T)qe[2], (T)qe[3], (T)qe[4],
                        (T)qe[5], (T)qe[6], (T)qe[7], (T)qe[8], (T)qe[9]};
}

// Terms of one QM-MM pair within the cutoff: offset (x, y, z) = site - atom
// (with its lattice image), r2 its squared length, q the MM charge.
//   BWD != 1: the 10 forward sums into acc[0..9] (phi, grad phi and half the
//             Hessian of phi at the site);
//   BWD != 0: dL/dR_site with the effective moments M into acc[OB..OB+2], and
//             with mm_side the MM atom's terms into mm[0..3]: the potential of
//             M per unit charge, and -q g.
template <typename T, int BWD>
DEV void pair_terms(T x, T y, T z, T r2, T q, T a, const SiteMoments<T>& M, double* acc, bool mm_side,
                    double (&mm)[4]) {
  constexpr int OB = BWD == 2 ? 10 : 0;
  const Radial<T> R = radial<T>(r2, a);
  if (BWD != 1) {
    acc[0] += (double)(q * R.f1);
    acc[1] += (double)(-q * x * R.f3);
    acc[2] += (double)(-q * y * R.f3);
    acc[3] += (double)(-q * z * R.f3);
    const T h5 = T(1.5) * q * R.f5, h3 = T(0.5) * q * R.f3;
    acc[4] += (double)(h5 * x * x - h3);
    acc[5] += (double)(h5 * x * y);
    acc[6] += (double)(h5 * x * z);
    acc[7] += (double)(h5 * y * y - h3);
    acc[8] += (double)(h5 * y * z);
    acc[9] += (double)(h5 * z * z - h3);
  }
  if (BWD != 0) {
    // g = Q psi1 + 2 mu.psi2 + 3 theta:psi3 (theta full symmetric)
    const T md = M.m0 * x + M.m1 * y + M.m2 * z;
    const T thx = M.t0 * x + M.t1 * y + M.t2 * z, thy = M.t1 * x + M.t3 * y + M.t4 * z,
            thz = M.t2 * x + M.t4 * y + M.t5 * z;
    const T dtd = x * thx + y * thy + z * thz;
    const T tr = M.t0 + M.t3 + M.t5;
    const T s1 = -M.Q * R.f3 + T(3) * md * R.f5 + T(1.5) * tr * R.f5 - T(7.5) * dtd * R.f7;
    const T s2 = -R.f3;
    const T s3 = T(3) * R.f5;
    const double gx = (double)(s1 * x + s2 * M.m0 + s3 * thx), gy = (double)(s1 * y + s2 * M.m1 + s3 * thy),
                 gz = (double)(s1 * z + s2 * M.m2 + s3 * thz);
    acc[OB + 0] += (double)q * gx;
    acc[OB + 1] += (double)q * gy;
    acc[OB + 2] += (double)q * gz;
    if (mm_side) {
      mm[0] = (double)(M.Q * R.f1 - md * R.f3 + T(1.5) * dtd * R.f5 - T(0.5) * tr * R.f3);
      mm[1] = -(double)q * gx;
      mm[2] = -(double)q * gy;
      mm[3] = -(double)q * gz;
    }
  }
}

// A wave's pair FIFO in LDS: x, y, z, r^2, q (T) and an atom index per entry.
template <typename T>
struct PairFifo {
  T *x, *y, *z, *r2, *q;
  int* idx;
  DEV PairFifo(void* lds, int wave) {
    x = reinterpret_cast<T*>(lds) + wave * 5 * kPairFifo;
    y = x + kPairFifo;
    z = y + kPairFifo;
    r2 = z + kPairFifo;
    q = r2 + kPairFifo;
    idx = reinterpret_cast<int*>(reinterpret_cast<T*>(lds) + 4 * 5 * kPairFifo) + wave * kPairFifo;
  }
  // append the hits of the wave's lanes, in lane order, after the count
  // pending entries; returns the new count (wave-uniform)
  DEV int append(bool hit, int lane, int count, double dx, double dy, double dz, double r2d, double qd, int i) {
    const unsigned long long mask = __ballot(hit);
    if (hit) {
      const int pos = count + (int)__popcll(mask & ((1ull << lane) - 1ull));
      x[pos] = (T)dx;
      y[pos] = (T)dy;
      z[pos] = (T)dz;
      r2[pos] = (T)r2d;
      q[pos] = (T)qd;
      idx[pos] = i;
    }
    return count + (int)__popcll(mask);
  }
  // after the first 64 entries were evaluated: move the remaining count - 64
  // (< 64) to the front; returns the new count
  DEV int drop64(int lane, int count) {
    T sx = 0, sy = 0, sz = 0, s2 = 0, sq = 0;
    int si = 0;
    const bool mv = lane < count - 64;
    if (mv) {
      sx = x[64 + lane];
      sy = y[64 + lane];
      sz = z[64 + lane];
      s2 = r2[64 + lane];
      sq = q[64 + lane];
      si = idx[64 + lane];
    }
    wave_lds_sync();
    if (mv) {
      x[lane] = sx;
      y[lane] = sy;
      z[lane] = sz;
      r2[lane] = s2;
      q[lane] = sq;
      idx[lane] = si;
    }
    return count - 64;
  }
};

// One item: QM site j of frame fr against MM chunk ci (of nchunk, chunk atoms
// each); red holds 4 x 13 doubles of LDS, fifo pair_fifo_bytes<T>() bytes.
template <typename T, int BWD>
DEV void real_qm_item(const Grid& g, const FrameDev& fr, int j, int ci, int nchunk, int chunk,
                      const double* __restrict__ qm4, int cap_qm, const double* __restrict__ mm4, int cap_mm,
                      const double* __restrict__ qeff, double* __restrict__ qacc, double* __restrict__ rpart,
                      double* __restrict__ det, double* red, void* fifo) {
  if (j >= fr.nq) return;
  const int i0 = ci * chunk;
  if (i0 >= fr.nm && !det) return;  // (with det every chunk writes its, possibly zero, partial sums)
  const int i1 = min(fr.nm, i0 + chunk);
  const int r = fr.qoff + j;
  const double X = qm4[r], Y = qm4[(size_t)cap_qm + r], Zc = qm4[(size_t)2 * cap_qm + r];
  const T a = (T)g.alpha;
  const double rc2 = g.rcut * g.rcut;
  // BWD: 0 forward (10 sums), 1 adjoint (3), 2 both (13).  With rpart (zeroed
  // beforehand) the adjoint also adds the MM-side terms of each pair.
  constexpr int NV = BWD == 0 ? 10 : BWD == 1 ? 3 : 13;
  constexpr int OB = BWD == 2 ? 10 : 0;
  double acc[NV];
#pragma unroll
  for (int t = 0; t < NV; t++) acc[t] = 0.0;
  const SiteMoments<T> M = BWD ? site_moments<T>(qeff + 10 * (size_t)r) : SiteMoments<T>{};
  const double* mx_ = mm4 + fr.moff;
  const double* my_ = mm4 + (size_t)cap_mm + fr.moff;
  const double* mz_ = mm4 + (size_t)2 * cap_mm + fr.moff;
  const double* mq_ = mm4 + (size_t)3 * cap_mm + fr.moff;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  PairFifo<T> ff(fifo, wave);
  // evaluate the first n (<= 64) pairs of the FIFO, one per lane
  auto evaluate = [&](int n) {
    if (lane >= n) return;
    double mm[4];
    pair_terms<T, BWD>(ff.x[lane], ff.y[lane], ff.z[lane], ff.r2[lane], ff.q[lane], a, M, acc, rpart != nullptr, mm);
    if (BWD != 0 && rpart) {
      double* o = rpart + (size_t)(fr.moff + ff.idx[lane]) * 4;
      for (int t = 0; t < 4; t++) atomicAdd(&o[t], mm[t]);
    }
  };
  int count = 0;  // pending pairs of this wave (wave-uniform)
  if (fr.nimg == 0) {
    // rc <= L/2 on every axis: the minimum image is a pair's only candidate
    // (the FIFO receives the same pairs in the same order as below)
    for (int base = i0; base < i1; base += 256) {  // rounds are uniform over the block
      const int i = base + threadIdx.x;
      double bx = 0.0, by = 0.0, bz = 0.0, qd = 0.0, r2d = 0.0;
      bool hit = false;
      if (i < i1) {
        bx = X - mx_[i];
        by = Y - my_[i];
        bz = Zc - mz_[i];
        qd = mq_[i];
        min_image(bx, by, bz, fr);
        r2d = bx * bx + by * by + bz * bz;
        hit = r2d < rc2 && r2d != 0.0;
      }
      count = ff.append(hit, lane, count, bx, by, bz, r2d, qd, i);
      if (count >= 64) {
        wave_lds_sync();
        evaluate(64);
        count = ff.drop64(lane, count);
      }
    }
  } else {
    for (int base = i0; base < i1; base += 256) {  // rounds are uniform over the block
      const int i = base + threadIdx.x;
      double bx = 0.0, by = 0.0, bz = 0.0, qd = 0.0;
      // this lane's candidate lattice images: per axis, the image offsets
      // whose distance along that axis can be within rc
      int lx = 0, hx = -1, ly = 0, hy = -1, lz = 0, hz = -1;
      if (i < i1) {
        bx = X - mx_[i];
        by = Y - my_[i];
        bz = Zc - mz_[i];
        qd = mq_[i];
        min_image(bx, by, bz, fr);
        image_range(bx, fr.box[0], fr.inv_box[0], g.rcut, fr.nimg, lx, hx);
        image_range(by, fr.box[1], fr.inv_box[1], g.rcut, fr.nimg, ly, hy);
        image_range(bz, fr.box[2], fr.inv_box[2], g.rcut, fr.nimg, lz, hz);
      }
      int ix_ = lx, iy_ = ly, iz_ = lz;
      bool more = lx <= hx && ly <= hy && lz <= hz;
      for (;;) {  // wave-uniform
        // test candidates until 64 pairs are pending or every lane is done
        // (the accumulators stay out of this loop)
        while (count < 64 && __ballot(more)) {
          bool hit = false;
          double dx = 0.0, dy = 0.0, dz = 0.0, r2d = 0.0;
          if (more) {
            dx = bx + ix_ * fr.box[0];
            dy = by + iy_ * fr.box[1];
            dz = bz + iz_ * fr.box[2];
            r2d = dx * dx + dy * dy + dz * dz;
            hit = r2d < rc2 && r2d != 0.0;
            if (++iz_ > hz) {
              iz_ = lz;
              if (++iy_ > hy) {
                iy_ = ly;
                more = ++ix_ <= hx;
              }
            }
          }
          count = ff.append(hit, lane, count, dx, dy, dz, r2d, qd, i);
        }
        if (count < 64) break;
        wave_lds_sync();
        evaluate(64);
        count = ff.drop64(lane, count);
      }
    }
  }
  wave_lds_sync();
  evaluate(count);
  double tot[NV];
  block_sum256_lds<NV>(acc, tot, red);
  if (threadIdx.x == 0 && det) {
    double* o = det + ((size_t)r * nchunk + ci) * 13;
    for (int t = 0; t < NV; t++) o[t] = tot[t];
  } else if (threadIdx.x == 0) {
    double* qa = qacc + (size_t)r * QA_STRIDE;
    if (BWD != 1) {
      atomicAdd(&qa[QA_PHI_SR], tot[0]);
      for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_DPHI_SR + t], tot[1 + t]);
      for (int t = 0; t < 6; t++) atomicAdd(&qa[QA_H_SR + t], tot[4 + t]);
    }
    if (BWD != 0)
      for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_G_QMMM_SR + t], tot[OB + t]);
  }
}

template <typename T, int BWD>
__global__ __launch_bounds__(256) void k_real_qm(Grid g, FrameArg fa, int chunk, const double* __restrict__ qm4,
                                                 int cap_qm, const double* __restrict__ mm4, int cap_mm,
                                                 const double* __restrict__ qeff, double* __restrict__ qacc,
                                                 double* __restrict__ rpart, double* __restrict__ det) {
  __shared__ double red[4 * 13];
  __shared__ __align__(16) char fifo[pair_fifo_bytes<T>()];
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  real_qm_item<T, BWD>(g, fr, blockIdx.x, blockIdx.y, gridDim.y, chunk, qm4, cap_qm, mm4, cap_mm, qeff, qacc, rpart,
                       det, red, fifo);
}

// Real space with lattice images (a cutoff beyond half a box length, where
// every (site, atom) pair has several images within it), forward and adjoint
// with both sides of each pair in one pass, so erfc and exp are evaluated once
// per pair.  A block takes 256 MM atoms and 4 * spw QM sites, each wave spw of
// them, site by site: the wave runs over the block's atoms 64 at a time,
// compacts the pairs within the cutoff into its LDS FIFO and evaluates them 64
// at a time, one per lane; at the end of a site it reduces the site's 13 sums
// over its lanes and adds them to the site's accumulator row.  The MM-side
// terms of each pair are added in LDS to the atom's four values, which go to
// rpart (zeroed beforehand) once per block.  No block barrier inside the site
// loop: waves with less work leave early.
template <typename T>
// (three waves per SIMD: 168 VGPRs with a few spilled, faster than two waves unspilled)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_real_img(Grid g, FrameArg fa, int spw, const double* __restrict__ qm4,
                                                  int cap_qm, const double* __restrict__ mm4, int cap_mm,
                                                  const double* __restrict__ qeff, double* __restrict__ qacc,
                                                  double* __restrict__ rpart) {
  __shared__ double mmacc[4 * 256];  // [term][atom of the block]
  __shared__ __align__(16) char fifo[pair_fifo_bytes<T>()];
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  const int a0 = blockIdx.x * 256, a1 = min(fr.nm, a0 + 256);
  if (a0 >= fr.nm || (int)blockIdx.y * 4 * spw >= fr.nq) return;  // block-uniform
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int t = 0; t < 4; t++) mmacc[t * 256 + tid] = 0.0;
  __syncthreads();
  const T a = (T)g.alpha;
  const double rc2 = g.rcut * g.rcut;
  const double* mx_ = mm4 + fr.moff;
  const double* my_ = mm4 + (size_t)cap_mm + fr.moff;
  const double* mz_ = mm4 + (size_t)2 * cap_mm + fr.moff;
  const double* mq_ = mm4 + (size_t)3 * cap_mm + fr.moff;
  PairFifo<T> ff(fifo, wave);
  const int jw0 = ((int)blockIdx.y * 4 + wave) * spw, jw1 = min(fr.nq, jw0 + spw);
  for (int j = jw0; j < jw1; j++) {  // wave-uniform
    const int r = fr.qoff + j;
    const double X = qm4[r], Y = qm4[(size_t)cap_qm + r], Zc = qm4[(size_t)2 * cap_qm + r];
    const SiteMoments<T> M = site_moments<T>(qeff + 10 * (size_t)r);
    double acc[13];
#pragma unroll
    for (int t = 0; t < 13; t++) acc[t] = 0.0;
    auto evaluate = [&](int n) {
      if (lane >= n) return;
      double mm[4];
      pair_terms<T, 2>(ff.x[lane], ff.y[lane], ff.z[lane], ff.r2[lane], ff.q[lane], a, M, acc, true, mm);
      const int k = ff.idx[lane];
      for (int t = 0; t < 4; t++) atomicAdd(&mmacc[t * 256 + k], mm[t]);
    };
    int count = 0;  // pending pairs of this wave (wave-uniform)
    for (int base = a0; base < a1; base += 64) {  // wave-uniform
      const int i = base + lane;
      double bx = 0.0, by = 0.0, bz = 0.0, qd = 0.0;
      int lx = 0, hx = -1, ly = 0, hy = -1, lz = 0, hz = -1;
      if (i < a1) {
        bx = X - mx_[i];
        by = Y - my_[i];
        bz = Zc - mz_[i];
        qd = mq_[i];
        min_image(bx, by, bz, fr);
        image_range(bx, fr.box[0], fr.inv_box[0], g.rcut, fr.nimg, lx, hx);
        image_range(by, fr.box[1], fr.inv_box[1], g.rcut, fr.nimg, ly, hy);
        image_range(bz, fr.box[2], fr.inv_box[2], g.rcut, fr.nimg, lz, hz);
      }
      int ix_ = lx, iy_ = ly, iz_ = lz;
      bool more = lx <= hx && ly <= hy && lz <= hz;
      for (;;) {  // wave-uniform
        // test candidates until 64 pairs are pending or every lane is done
        // (the accumulators stay out of this loop)
        while (count < 64 && __ballot(more)) {
          bool hit = false;
          double dx = 0.0, dy = 0.0, dz = 0.0, r2d = 0.0;
          if (more) {
            dx = bx + ix_ * fr.box[0];
            dy = by + iy_ * fr.box[1];
            dz = bz + iz_ * fr.box[2];
            r2d = dx * dx + dy * dy + dz * dz;
            hit = r2d < rc2 && r2d != 0.0;
            if (++iz_ > hz) {
              iz_ = lz;
              if (++iy_ > hy) {
                iy_ = ly;
                more = ++ix_ <= hx;
              }
            }
          }
          count = ff.append(hit, lane, count, dx, dy, dz, r2d, qd, i - a0);
        }
        if (count < 64) break;
        wave_lds_sync();
        evaluate(64);
        count = ff.drop64(lane, count);
      }
    }
    wave_lds_sync();
    evaluate(count);
    wave_lds_sync();  // the FIFO is refilled from the front for the next site
#pragma unroll
    for (int t = 0; t < 13; t++) acc[t] = wave_sum(acc[t]);
    if (lane == 0) {
      double* qa = qacc + (size_t)r * QA_STRIDE;
      atomicAdd(&qa[QA_PHI_SR], acc[0]);
      for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_DPHI_SR + t], acc[1 + t]);
      for (int t = 0; t < 6; t++) atomicAdd(&qa[QA_H_SR + t], acc[4 + t]);
      for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_G_QMMM_SR + t], acc[10 + t]);
    }
  }
  __syncthreads();  // every wave's LDS adds are done
  if (a0 + tid < a1) {
    double* o = rpart + (size_t)(fr.moff + a0 + tid) * 4;
    for (int t = 0; t < 4; t++) atomicAdd(&o[t], mmacc[t * 256 + tid]);
  }
}

// waves the lattice-image kernel aims for (sites per wave are sized to reach it)
static constexpr long kImgWaves = 4096;

hipError_t launch_real_img(const Grid& g, const FrameArg& fa, int max_nq, int max_nm, int cap_qm, int cap_mm,
                           int fp32, Work& w, hipStream_t s) {
  const int bx = (max_nm + 255) / 256;
  const long site_waves = (long)bx * fa.n_frames * max_nq;  // waves at one site each
  const int spw = (int)std::max(1L, site_waves / kImgWaves);
  dim3 grid(bx, (max_nq + 4 * spw - 1) / (4 * spw), fa.n_frames);
  if (fp32)
    hipLaunchKernelGGL(k_real_img<float>, grid, dim3(256), 0, s, g, fa, spw, w.qm4, cap_qm, w.mm4, cap_mm, w.qeff,
                       w.qacc, w.rpart);
  else
    hipLaunchKernelGGL(k_real_img<double>, grid, dim3(256), 0, s, g, fa, spw, w.qm4, cap_qm, w.mm4, cap_mm, w.qeff,
                       w.qacc, w.rpart);
  return hipGetLastError();
}

static constexpr int kRealChunk = 2048;

hipError_t launch_real_qm(const Grid& g, const FrameArg& fa, int max_nq, int max_nm, int cap_qm, int cap_mm,
                          int backward, int fp32, Work& w, hipStream_t s, double* rpart, int mm_groups) {
  if (max_nq == 0 || max_nm == 0) return hipSuccess;
  // lattice images, forward and adjoint with the MM side: one pass over each
  // pair for both sides (deterministic plans keep the fixed-order kernels)
  if (backward == 2 && rpart && mm_groups > 0 && !w.det_real)
    return launch_real_img(g, fa, max_nq, max_nm, cap_qm, cap_mm, fp32, w, s);
  // with lattice images (mm_groups > 0) a (site, atom) pair tests up to 8
  // images: smaller chunks keep enough blocks in flight
  int chunk = mm_groups > 0 ? kRealChunk / 4 : kRealChunk;
  double* det = w.det_real;
  if (det) {
    // at most kDetChunks partial rows per site; the MM-side terms come from
    // the per-atom kernel (fixed order over the sites) instead of atomics
    chunk = max(chunk, ((max_nm + kDetChunks - 1) / kDetChunks + 255) / 256 * 256);
  }
  // MM-side terms: per pair into rpart from this kernel, or (deterministic
  // mode, or mm_groups > 0) from the per-atom kernel afterwards
  const bool per_atom = rpart && backward && (det || mm_groups > 0);
  double* rp = per_atom ? (double*)nullptr : rpart;
  dim3 grid(max_nq, (max_nm + chunk - 1) / chunk, fa.n_frames);
#define RQ(T, B)                                                                                              \
  hipLaunchKernelGGL((k_real_qm<T, B>), grid, dim3(256), 0, s, g, fa, chunk, w.qm4, cap_qm, w.mm4, cap_mm, \
                     w.qeff, w.qacc, rp, det)
  if (fp32) {
    if (backward == 2) RQ(float, 2); else if (backward) RQ(float, 1); else RQ(float, 0);
  } else {
    if (backward == 2) RQ(double, 2); else if (backward) RQ(double, 1); else RQ(double, 0);
  }
#undef RQ
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (det) {
    DetMap m{};
    if (backward != 1) m = det_range(m, QA_PHI_SR, 10);
    if (backward) m = det_range(m, QA_G_QMMM_SR, 3);
    e = launch_det_reduce(fa, 1, max_nq, det, (int)grid.y, 13, m, w.qacc, QA_STRIDE, s);
    if (e != hipSuccess) return e;
  }
  if (!per_atom) return hipSuccess;
  // one site group writes each atom's terms in a fixed order (deterministic);
  // several add into rpart, which prep zeroed
  return launch_real_mm(g, fa, max_nq, max_nm, cap_qm, cap_mm, fp32, w, s, det ? 1 : mm_groups);
}

// MM side of the QM-MM real-space sum (backward): dL/dR_i and dL/dq_i with
// the effective moments, one thread per MM atom looping over the QM sites of
// its block's site group (blockIdx.y of gridDim.y groups), for each site over
// the lattice images whose per-axis offsets can lie within the cutoff.  With
// one group the thread writes its atom's four values; with several (the
// paper's rc ~ L regime, where the per-atom work is large) it adds them to
// rpart, which the caller has zeroed.
template <typename T>
__global__ __launch_bounds__(256) void k_real_mm(Grid g, FrameArg fa, const double* __restrict__ qm4, int cap_qm,
                                                 const double* __restrict__ mm4, int cap_mm,
                                                 const double* __restrict__ qeff, double* __restrict__ rpart,
                                                 int sites_per_group) {
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= fr.nm) return;
  const int j0 = blockIdx.y * sites_per_group, j1 = min(fr.nq, j0 + sites_per_group);
  if (j0 >= j1 && gridDim.y > 1) return;  // (one group: the atom's zero terms are still written)
  const int row = fr.moff + i;
  const double X = mm4[row], Y = mm4[(size_t)cap_mm + row], Zc = mm4[(size_t)2 * cap_mm + row];
  const double q = mm4[(size_t)3 * cap_mm + row];
  const T a = (T)g.alpha;
  const double rc2 = g.rcut * g.rcut;
  double aphi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int j = j0; j < j1; j++) {
    const int r = fr.qoff + j;
    double bx = qm4[r] - X, by = qm4[(size_t)cap_qm + r] - Y, bz = qm4[(size_t)2 * cap_qm + r] - Zc;
    min_image(bx, by, bz, fr);
    int lx, hx, ly, hy, lz, hz;
    image_range(bx, fr.box[0], fr.inv_box[0], g.rcut, fr.nimg, lx, hx);
    image_range(by, fr.box[1], fr.inv_box[1], g.rcut, fr.nimg, ly, hy);
    image_range(bz, fr.box[2], fr.inv_box[2], g.rcut, fr.nimg, lz, hz);
    for (int ix_ = lx; ix_ <= hx; ix_++)
      for (int iy_ = ly; iy_ <= hy; iy_++)
        for (int iz_ = lz; iz_ <= hz; iz_++) {
          const double dx = bx + ix_ * fr.box[0], dy = by + iy_ * fr.box[1], dz = bz + iz_ * fr.box[2];
          const double r2d = dx * dx + dy * dy + dz * dz;
          if (!(r2d < rc2) || r2d == 0.0) continue;
          const T x = (T)dx, y = (T)dy, z = (T)dz;
          const Radial<T> R = radial<T>((T)r2d, a);
          const double* qe = qeff + 10 * (size_t)r;
          const T Qe = (T)qe[0], m0 = (T)qe[1], m1 = (T)qe[2], m2 = (T)qe[3];
          const T t0 = (T)qe[4], t1 = (T)qe[5], t2 = (T)qe[6], t3 = (T)qe[7], t4 = (T)qe[8], t5 = (T)qe[9];
          const T md = m0 * x + m1 * y + m2 * z;
          const T thx = t0 * x + t1 * y + t2 * z, thy = t1 * x + t3 * y + t4 * z, thz = t2 * x + t4 * y + t5 * z;
          const T dtd = x * thx + y * thy + z * thz;
          const T tr = t0 + t3 + t5;
          // energy per unit MM charge: Q psi0 + mu.psi1 + theta:psi2
          aphi += (double)(Qe * R.f1 - md * R.f3 + T(1.5) * dtd * R.f5 - T(0.5) * tr * R.f3);
          const T s1 = -Qe * R.f3 + T(3) * md * R.f5 + T(1.5) * tr * R.f5 - T(7.5) * dtd * R.f7;
          const T s2 = -R.f3;
          const T s3 = T(3) * R.f5;
          // r depends on -R_mm
          gx -= (double)(s1 * x + s2 * m0 + s3 * thx);
          gy -= (double)(s1 * y + s2 * m1 + s3 * thy);
          gz -= (double)(s1 * z + s2 * m2 + s3 * thz);
        }
  }
  double* o = rpart + (size_t)row * 4;
  if (gridDim.y == 1) {
    o[0] = aphi;
    o[1] = q * gx;
    o[2] = q * gy;
    o[3] = q * gz;
  } else {
    atomicAdd(&o[0], aphi);
    atomicAdd(&o[1], q * gx);
    atomicAdd(&o[2], q * gy);
    atomicAdd(&o[3], q * gz);
  }
}

hipError_t launch_real_mm(const Grid& g, const FrameArg& fa, int max_nq, int max_nm, int cap_qm, int cap_mm,
                          int fp32, Work& w, hipStream_t s, int groups) {
  if (max_nm == 0) return hipSuccess;
  if (groups < 1 || max_nq <= 1) groups = 1;
  if (groups > max_nq) groups = max_nq;
  const int spg = (max_nq + groups - 1) / groups;
  groups = (max_nq + spg - 1) / spg;
  dim3 grid((max_nm + 255) / 256, groups, fa.n_frames);
  if (fp32)
    hipLaunchKernelGGL(k_real_mm<float>, grid, dim3(256), 0, s, g, fa, w.qm4, cap_qm, w.mm4, cap_mm, w.qeff, w.rpart,
                       spg);
  else
    hipLaunchKernelGGL(k_real_mm<double>, grid, dim3(256), 0, s, g, fa, w.qm4, cap_qm, w.mm4, cap_mm, w.qeff, w.rpart,
                       spg);
  return hipGetLastError();
}

// ------------------------------------------------------------------ cell list
// MM atoms are binned into nc[0] x nc[1] x nc[2] cells of edge >= rcut (at
// least 3 per axis), so all minimum-image partners within rcut of a point lie
// in its cell and the 26 around it.  Counting sort: count, scan, fill.
// Cell index along one axis of a wrapped coordinate, clamped to [0, n - 1]
// at both ends before the conversion; a NaN coordinate (NaN input) lands in
// cell 0, so no index ever leaves the cell arrays.
DEV int cell_axis(double x, double inv_box, int n) {
  const double c = x * inv_box * (double)n;
  return c >= 0.0 ? (c < (double)(n - 1) ? (int)c : n - 1) : 0;
}

DEV int cell_of(double x, double y, double z, const FrameDev& fr) {
  const int cx = cell_axis(x, fr.inv_box[0], fr.nc[0]);
  const int cy = cell_axis(y, fr.inv_box[1], fr.nc[1]);
  const int cz = cell_axis(z, fr.inv_box[2], fr.nc[2]);
  return (cx * fr.nc[1] + cy) * fr.nc[2] + cz;
}

// block-local histogram in LDS, one global atomic per (block, occupied cell)
__global__ __launch_bounds__(256) void k_cell_count(FrameArg fa, const double* __restrict__ mm4, int cap_mm,
                                                    int* __restrict__ cell_cnt, int* __restrict__ atom_cell) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  if (fr.nc[0] == 0 || blockIdx.x * 256 >= fr.nm) return;
  const int ncell = fr.nc[0] * fr.nc[1] * fr.nc[2];
  __shared__ int hist[kMaxCellsPerAxis * kMaxCellsPerAxis * kMaxCellsPerAxis];
  for (int c = threadIdx.x; c < ncell; c += 256) hist[c] = 0;
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < fr.nm) {
    const int row = fr.moff + i;
    const int c = cell_of(mm4[row], mm4[(size_t)cap_mm + row], mm4[(size_t)2 * cap_mm + row], fr);
    atom_cell[row] = c;
    atomicAdd(&hist[c], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncell; c += 256)
    if (hist[c]) atomicAdd(&cell_cnt[fr.cell_base + c], hist[c]);
}

// one block per frame: exclusive scan of the counts (ncells + 1 entries), counts reset for the fill
__global__ __launch_bounds__(256) void k_cell_scan(FrameArg fa, int* __restrict__ cell_cnt,
                                                   int* __restrict__ cell_start) {
  const int f = blockIdx.x;
  const FrameDev fr = get_frame(fa, f);
  if (fr.nc[0] == 0) return;
  const int n = fr.nc[0] * fr.nc[1] * fr.nc[2];
  const int per = (n + 255) / 256;
  const int b0 = threadIdx.x * per, b1 = min(n, b0 + per);
  int local = 0;
  for (int c = b0; c < b1; c++) local += cell_cnt[fr.cell_base + c];
  __shared__ int part[256];
  part[threadIdx.x] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < 256; t++) {
      const int v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int c = b0; c < b1; c++) {
    const int v = cell_cnt[fr.cell_base + c];
    cell_start[fr.cell_base + c] = run;
    cell_cnt[fr.cell_base + c] = 0;
    run += v;
  }
  if (threadIdx.x == 255) cell_start[fr.cell_base + n] = fr.nm;
}

// ranks within the block from LDS atomics, one global atomic per (block, cell) for the base
__global__ __launch_bounds__(256) void k_cell_fill(FrameArg fa, int* __restrict__ cell_cnt,
                                                   const int* __restrict__ cell_start,
                                                   const int* __restrict__ atom_cell, int* __restrict__ cell_atoms) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  if (fr.nc[0] == 0 || blockIdx.x * 256 >= fr.nm) return;
  const int ncell = fr.nc[0] * fr.nc[1] * fr.nc[2];
  __shared__ int cnt[kMaxCellsPerAxis * kMaxCellsPerAxis * kMaxCellsPerAxis];
  for (int c = threadIdx.x; c < ncell; c += 256) cnt[c] = 0;
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  int c = -1, rank = 0;
  if (i < fr.nm) {
    c = atom_cell[fr.moff + i];
    rank = atomicAdd(&cnt[c], 1);
  }
  __syncthreads();
  for (int cc = threadIdx.x; cc < ncell; cc += 256)
    if (cnt[cc]) cnt[cc] = atomicAdd(&cell_cnt[fr.cell_base + cc], cnt[cc]);
  __syncthreads();
  if (c >= 0) cell_atoms[fr.moff + cell_start[fr.cell_base + c] + cnt[c] + rank] = i;
}

hipError_t launch_cells(const FrameArg& fa, int max_nm, int cap_mm, Work& w, hipStream_t s) {
  if (max_nm == 0) return hipSuccess;
  dim3 grid((max_nm + 255) / 256, fa.n_frames);
  hipLaunchKernelGGL(k_cell_count, grid, dim3(256), 0, s, fa, w.mm4, cap_mm, w.cell_cnt, w.atom_cell);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_scan, dim3(fa.n_frames), dim3(256), 0, s, fa, w.cell_cnt, w.cell_start);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_fill, grid, dim3(256), 0, s, fa, w.cell_cnt, w.cell_start, w.atom_cell, w.cell_atoms);
  return hipGetLastError();
}

// Real space over the cell list: block (QM site, one of the 27 neighbour
// cells).  Forward accumulates phi, grad phi, 1/2 grad grad phi of the site;
// backward accumulates dL/dR of the site (effective moments) and adds the MM
// partners' dL/dR and dL/dq into rpart.
template <typename T, int BWD>
__global__ __launch_bounds__(256) void k_real_cells(Grid g, FrameArg fa, const double* __restrict__ qm4, int cap_qm,
                                                    const double* __restrict__ mm4, int cap_mm,
                                                    const int* __restrict__ cell_start,
                                                    const int* __restrict__ cell_atoms,
                                                    const double* __restrict__ qeff, double* __restrict__ qacc,
                                                    double* __restrict__ rpart) {
  const int f = blockIdx.z;
  const FrameDev fr = get_frame(fa, f);
  const int j = blockIdx.x;
  if (j >= fr.nq) return;
  const int r = fr.qoff + j;
  const double X = qm4[r], Y = qm4[(size_t)cap_qm + r], Zc = qm4[(size_t)2 * cap_qm + r];
  // neighbour cell of this block
  const int nb = blockIdx.y;
  const int dx = nb / 9 - 1, dy = (nb / 3) % 3 - 1, dz = nb % 3 - 1;
  const int cx = cell_axis(X, fr.inv_box[0], fr.nc[0]);
  const int cy = cell_axis(Y, fr.inv_box[1], fr.nc[1]);
  const int cz = cell_axis(Zc, fr.inv_box[2], fr.nc[2]);
  const int c = (((cx + dx + fr.nc[0]) % fr.nc[0]) * fr.nc[1] + (cy + dy + fr.nc[1]) % fr.nc[1]) * fr.nc[2] +
                (cz + dz + fr.nc[2]) % fr.nc[2];
  const int s0 = cell_start[fr.cell_base + c], s1 = cell_start[fr.cell_base + c + 1];
  const T a = (T)g.alpha;
  const double rc2 = g.rcut * g.rcut;
  constexpr int NV = BWD ? 3 : 10;
  double acc[NV];
#pragma unroll
  for (int t = 0; t < NV; t++) acc[t] = 0.0;
  T Qe = 0, m0 = 0, m1 = 0, m2 = 0, t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0, t5 = 0;
  if (BWD) {
    const double* qe = qeff + 10 * (size_t)r;
    Qe = (T)qe[0]; m0 = (T)qe[1]; m1 = (T)qe[2]; m2 = (T)qe[3];
    t0 = (T)qe[4]; t1 = (T)qe[5]; t2 = (T)qe[6]; t3 = (T)qe[7]; t4 = (T)qe[8]; t5 = (T)qe[9];
  }
  for (int p = s0 + threadIdx.x; p < s1; p += 256) {
    const int i = cell_atoms[fr.moff + p];
    const int row = fr.moff + i;
    double ddx = X - mm4[row], ddy = Y - mm4[(size_t)cap_mm + row], ddz = Zc - mm4[(size_t)2 * cap_mm + row];
    min_image(ddx, ddy, ddz, fr);
    const double r2d = ddx * ddx + ddy * ddy + ddz * ddz;
    if (!(r2d < rc2) || r2d == 0.0) continue;
    const T x = (T)ddx, y = (T)ddy, z = (T)ddz;
    const Radial<T> R = radial<T>((T)r2d, a);
    const T q = (T)mm4[(size_t)3 * cap_mm + row];
    if (!BWD) {
      acc[0] += (double)(q * R.f1);
      acc[1] += (double)(-q * x * R.f3);
      acc[2] += (double)(-q * y * R.f3);
      acc[3] += (double)(-q * z * R.f3);
      const T h5 = T(1.5) * q * R.f5, h3 = T(0.5) * q * R.f3;
      acc[4] += (double)(h5 * x * x - h3);
      acc[5] += (double)(h5 * x * y);
      acc[6] += (double)(h5 * x * z);
      acc[7] += (double)(h5 * y * y - h3);
      acc[8] += (double)(h5 * y * z);
      acc[9] += (double)(h5 * z * z - h3);
    } else {
      const T md = m0 * x + m1 * y + m2 * z;
      const T thx = t0 * x + t1 * y + t2 * z, thy = t1 * x + t3 * y + t4 * z, thz = t2 * x + t4 * y + t5 * z;
      const T dtd = x * thx + y * thy + z * thz;
      const T tr = t0 + t3 + t5;
      const T s1c = -Qe * R.f3 + T(3) * md * R.f5 + T(1.5) * tr * R.f5 - T(7.5) * dtd * R.f7;
      const T s2 = -R.f3;
      const T s3 = T(3) * R.f5;
      const double gx = (double)(s1c * x + s2 * m0 + s3 * thx), gy = (double)(s1c * y + s2 * m1 + s3 * thy),
                   gz = (double)(s1c * z + s2 * m2 + s3 * thz);
      acc[0] += (double)q * gx;
      acc[1] += (double)q * gy;
      acc[2] += (double)q * gz;
      double* o = rpart + (size_t)row * 4;
      atomicAdd(&o[0], (double)(Qe * R.f1 - md * R.f3 + T(1.5) * dtd * R.f5 - T(0.5) * tr * R.f3));
      atomicAdd(&o[1], -(double)q * gx);
      atomicAdd(&o[2], -(double)q * gy);
      atomicAdd(&o[3], -(double)q * gz);
    }
  }
  double tot[NV];
  block_sum256<NV>(acc, tot);
  if (threadIdx.x == 0) {
    double* qa = qacc + (size_t)r * QA_STRIDE;
    if (!BWD) {
      atomicAdd(&qa[QA_PHI_SR], tot[0]);
      for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_DPHI_SR + t], tot[1 + t]);
      for (int t = 0; t < 6; t++) atomicAdd(&qa[QA_H_SR + t], tot[4 + t]);
    } else {
      for (int t = 0; t < 3; t++) atomicAdd(&qa[QA_G_QMMM_SR + t], tot[t]);
    }
  }
}

hipError_t launch_real_cells(const Grid& g, const FrameArg& fa, int max_nq, int cap_qm, int cap_mm, int backward,
                             int fp32, Work& w, hipStream_t s) {
  if (max_nq == 0) return hipSuccess;
  dim3 grid(max_nq, 27, fa.n_frames);
#define RC(T, B)                                                                                                  \
  hipLaunchKernelGGL((k_real_cells<T, B>), grid, dim3(256), 0, s, g, fa, w.qm4, cap_qm, w.mm4, cap_mm,           \
                     w.cell_start, w.cell_atoms, w.qeff, w.qacc, w.rpart)
  if (fp32) {
    if (backward) RC(float, 1); else RC(float, 0);
  } else {
    if (backward) RC(double, 1); else RC(double, 0);
  }
#undef RC
  return hipGetLastError();
}

// ------------------------------------------------------------------ QM-QM real space, self, background
// P(a,b) = Qa Qb psi0 + (Qb mu_a - Qa mu_b).psi1 + (Qb th_a + Qa th_b):psi2 - 2 mu_a.psi2.mu_b,
// E = 1/2 sum_{a != b} P + sum_a self_a - (pi/(2 a^2 V)) Qtot^2.  One block per
// site a; its threads take the partners b and the block sums the site's
// energy share, position gradient and moment derivatives.
// One item: QM site a of frame f; red holds 4 x 14 doubles of LDS.
DEV void qmqm_item(const Grid& g, const FrameDev& fr, int f, int a, const double* __restrict__ qm4, int cap_qm,
                   const double* __restrict__ Q, const double* __restrict__ mu, const double* __restrict__ theta,
                   double* __restrict__ qacc, double* __restrict__ facc, double* __restrict__ det, double* red) {
  if (a >= fr.nq) return;
  const double al = g.alpha, rc2 = g.rcut * g.rcut;
  const double sp = 1.7724538509055160273;  // sqrt(pi)
  const double V = fr.box[0] * fr.box[1] * fr.box[2];
  const double bgc = -g.bgw * kPi / (al * al * V);
  const double Qtot = facc[f * FA_COUNT + FA_QTOT_QM];
  const int ra = fr.qoff + a;
  const double Xa = qm4[ra], Ya = qm4[(size_t)cap_qm + ra], Za = qm4[(size_t)2 * cap_qm + ra];
  const double Qa = Q[ra];
  const double ma0 = mu[3 * (size_t)ra], ma1 = mu[3 * (size_t)ra + 1], ma2 = mu[3 * (size_t)ra + 2];
  const double* tha = theta + 6 * (size_t)ra;
  // e, g0..2, dQ, dm0..2, dt0..5
  double v[14];
  for (int t = 0; t < 14; t++) v[t] = 0.0;
  for (int b = threadIdx.x; b < fr.nq; b += 256) {
    // a site's own images count when the cutoff exceeds the box (r = 0 is excluded below)
    if (b == a && fr.nimg == 0) continue;
    const int rb = fr.qoff + b;
    double bx = Xa - qm4[rb], by = Ya - qm4[(size_t)cap_qm + rb], bz = Za - qm4[(size_t)2 * cap_qm + rb];
    min_image(bx, by, bz, fr);
    const int n1_ = 2 * fr.nimg + 1;
    for (int im_ = 0; im_ < n1_ * n1_ * n1_; im_++) {
      // lattice images within the cutoff (only the minimum image when rc <= L/2)
      const int ix_ = im_ / (n1_ * n1_) - fr.nimg, iy_ = (im_ / n1_) % n1_ - fr.nimg, iz_ = im_ % n1_ - fr.nimg;
      const double x = bx + ix_ * fr.box[0], y = by + iy_ * fr.box[1], z = bz + iz_ * fr.box[2];
      const double r2 = x * x + y * y + z * z;
      if (!(r2 < rc2) || r2 == 0.0) continue;
      const Radial<double> R = radial<double>(r2, al);
      const double Qb = Q[rb];
      const double mb0 = mu[3 * (size_t)rb], mb1 = mu[3 * (size_t)rb + 1], mb2 = mu[3 * (size_t)rb + 2];
      const double* thb = theta + 6 * (size_t)rb;
      const double c0 = Qb * ma0 - Qa * mb0, c1 = Qb * ma1 - Qa * mb1, c2 = Qb * ma2 - Qa * mb2;
      double sm[6];
      for (int t = 0; t < 6; t++) sm[t] = Qb * tha[t] + Qa * thb[t];
      const double cd = c0 * x + c1 * y + c2 * z;
      const double sx = sm[0] * x + sm[1] * y + sm[2] * z, sy = sm[1] * x + sm[3] * y + sm[4] * z,
                   sz = sm[2] * x + sm[4] * y + sm[5] * z;
      const double dsd = x * sx + y * sy + z * sz, trs = sm[0] + sm[3] + sm[5];
      const double mad = ma0 * x + ma1 * y + ma2 * z, mbd = mb0 * x + mb1 * y + mb2 * z;
      const double mab = ma0 * mb0 + ma1 * mb1 + ma2 * mb2;
      const double P = Qa * Qb * R.f1 - cd * R.f3 + (1.5 * dsd * R.f5 - 0.5 * trs * R.f3) -
                       (3.0 * mad * mbd * R.f5 - mab * R.f3);
      v[0] += 0.5 * P;
      // dP/dr = QaQb psi1 + 2 c.psi2 + 3 s:psi3 - 6 mu_a.psi3.mu_b
      const double s1 = -Qa * Qb * R.f3 + 3.0 * cd * R.f5 + 1.5 * trs * R.f5 - 7.5 * dsd * R.f7 -
                        3.0 * (mab * R.f5 - 5.0 * mad * mbd * R.f7);
      const double sc = -R.f3, ss = 3.0 * R.f5, smu = -3.0 * R.f5;
      v[1] += s1 * x + sc * c0 + ss * sx + smu * (ma0 * mbd + mb0 * mad);
      v[2] += s1 * y + sc * c1 + ss * sy + smu * (ma1 * mbd + mb1 * mad);
      v[3] += s1 * z + sc * c2 + ss * sz + smu * (ma2 * mbd + mb2 * mad);
      const double thbx = thb[0] * x + thb[1] * y + thb[2] * z, thby = thb[1] * x + thb[3] * y + thb[4] * z,
                   thbz = thb[2] * x + thb[4] * y + thb[5] * z;
      const double dtbd = x * thbx + y * thby + z * thbz, trb = thb[0] + thb[3] + thb[5];
      v[4] += Qb * R.f1 + mbd * R.f3 + (1.5 * dtbd * R.f5 - 0.5 * trb * R.f3);
      v[5] += -Qb * x * R.f3 - (3.0 * x * mbd * R.f5 - mb0 * R.f3);
      v[6] += -Qb * y * R.f3 - (3.0 * y * mbd * R.f5 - mb1 * R.f3);
      v[7] += -Qb * z * R.f3 - (3.0 * z * mbd * R.f5 - mb2 * R.f3);
      const double h5 = 1.5 * Qb * R.f5, h3 = 0.5 * Qb * R.f3;
      v[8] += h5 * x * x - h3;
      v[9] += h5 * x * y;
      v[10] += h5 * x * z;
      v[11] += h5 * y * y - h3;
      v[12] += h5 * y * z;
      v[13] += h5 * z * z - h3;
    }
  }
  double tot[14];
  block_sum256_lds<14>(v, tot, red);
  if (threadIdx.x == 0) {
    // self terms of site a
    const double a3 = 2.0 * al * al * al / (3.0 * sp);
    const double tra = tha[0] + tha[3] + tha[5];
    const double mm2 = ma0 * ma0 + ma1 * ma1 + ma2 * ma2;
    double e = tot[0] - al / sp * Qa * Qa - a3 * mm2 + a3 * Qa * tra;
    if (a == 0) e += 0.5 * bgc * Qtot * Qtot;
    double* qa = qacc + (size_t)ra * QA_STRIDE;
    for (int t = 0; t < 3; t++) qa[QA_G_QQ_SR + t] = tot[1 + t];
    qa[QA_DQ_QQ_SR] = tot[4] - 2.0 * al / sp * Qa + a3 * tra + bgc * Qtot;
    for (int t = 0; t < 3; t++) qa[QA_DMU_QQ_SR + t] = tot[5 + t] - 2.0 * a3 * (t == 0 ? ma0 : t == 1 ? ma1 : ma2);
    for (int t = 0; t < 6; t++) qa[QA_DTH_QQ_SR + t] = tot[8 + t] + ((t == 0 || t == 3 || t == 5) ? a3 * Qa : 0.0);
    if (det)
      det[ra] = e;
    else
      atomicAdd(&facc[f * FA_COUNT + FA_E_QQ_SR], e);
  }
}

__global__ __launch_bounds__(256) void k_qmqm(Grid g, FrameArg fa, const double* __restrict__ qm4, int cap_qm,
                                              const double* __restrict__ Q, const double* __restrict__ mu,
                                              const double* __restrict__ theta, double* __restrict__ qacc,
                                              double* __restrict__ facc, double* __restrict__ det) {
  __shared__ double red[4 * 14];
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  qmqm_item(g, fr, f, blockIdx.x, qm4, cap_qm, Q, mu, theta, qacc, facc, det, red);
}

hipError_t launch_qmqm(const Grid& g, const FrameArg& fa, int max_nq, int cap_qm, const double* Q, const double* mu,
                       const double* theta, Work& w, hipStream_t s) {
  if (max_nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qmqm, dim3(max_nq, fa.n_frames), dim3(256), 0, s, g, fa, w.qm4, cap_qm, Q, mu, theta, w.qacc,
                     w.facc, w.det_qq);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !w.det_qq) return e;
  return launch_det_reduce(fa, 2, 1, w.det_qq, 0, 1, det_map({FA_E_QQ_SR}), w.facc, FA_COUNT, s);
}

// ------------------------------------------------------------------ forward outputs
// phi = SR + LR + background of the MM charges; E = sum_j [Q phi + mu.grad phi
// + theta:(1/2 grad grad phi)] + E_QQ.  One block per frame.
__global__ __launch_bounds__(256) void k_finalize_fwd(Grid g, FrameArg fa, const double* __restrict__ Q,
                                                      const double* __restrict__ mu,
                                                      const double* __restrict__ theta, int qmqm,
                                                      const double* __restrict__ qacc,
                                                      const double* __restrict__ facc, double* __restrict__ energy,
                                                      double* __restrict__ phi, double* __restrict__ efield,
                                                      double* __restrict__ efgrad, double* __restrict__ site) {
  const int f = blockIdx.x;
  const FrameDev fr = get_frame(fa, f);
  const double V = fr.box[0] * fr.box[1] * fr.box[2];
  const double bg = -g.bgw * kPi / (g.alpha * g.alpha * V) * facc[f * FA_COUNT + FA_QTOT_MM];
  double esum = 0.0;
  for (int j = threadIdx.x; j < fr.nq; j += 256) {
    const int r = fr.qoff + j;
    const double* qa = qacc + (size_t)r * QA_STRIDE;
    const double p = qa[QA_PHI_SR] + qa[QA_PHI_LR] + bg;
    double d[3], h[6];
    for (int t = 0; t < 3; t++) d[t] = qa[QA_DPHI_SR + t] + qa[QA_DPHI_LR + t];
    for (int t = 0; t < 6; t++) h[t] = qa[QA_H_SR + t] + qa[QA_H_LR + t];
    if (phi) phi[r] = p;
    if (efield)
      for (int t = 0; t < 3; t++) efield[3 * (size_t)r + t] = -d[t];
    if (efgrad)
      for (int t = 0; t < 6; t++) efgrad[6 * (size_t)r + t] = -2.0 * h[t];
    if (site) {
      double* o = site + 10 * (size_t)r;
      o[0] = p;
      for (int t = 0; t < 3; t++) o[1 + t] = d[t];
      for (int t = 0; t < 6; t++) o[4 + t] = h[t];
    }
    const double* m = mu + 3 * (size_t)r;
    const double* th = theta + 6 * (size_t)r;
    esum += Q[r] * p + m[0] * d[0] + m[1] * d[1] + m[2] * d[2] + th[0] * h[0] + th[3] * h[3] + th[5] * h[5] +
            2.0 * (th[1] * h[1] + th[2] * h[2] + th[4] * h[4]);
  }
  double v[1] = {esum}, tot[1];
  block_sum256<1>(v, tot);
  if (threadIdx.x == 0) {
    double e = tot[0];
    if (qmqm) e += facc[f * FA_COUNT + FA_E_QQ_LR] + facc[f * FA_COUNT + FA_E_QQ_SR];
    energy[fr.orig] = e;
  }
}

hipError_t launch_finalize_fwd(const Grid& g, const FrameArg& fa, const double* Q, const double* mu,
                               const double* theta, int qmqm, double* energy, double* phi, double* efield,
                               double* efgrad, double* site_out, Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_fwd, dim3(fa.n_frames), dim3(256), 0, s, g, fa, Q, mu, theta, qmqm, w.qacc, w.facc,
                     energy, phi, efield, efgrad, site_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ backward helpers
// Effective moments: L = gE E + g_phi.phi + g_efield.efield + g_efgrad.efgrad
// enters the QM-MM coupling exactly like E with Q' = gE Q + g_phi,
// mu' = gE mu - g_efield, theta'(stored) = gE theta - (2,1,1,2,1,2) * g_efgrad.
__global__ __launch_bounds__(256) void k_eff_moments(FrameArg fa, const double* __restrict__ Q,
                                                     const double* __restrict__ mu, const double* __restrict__ theta,
                                                     const double* __restrict__ gE, const double* __restrict__ g_phi,
                                                     const double* __restrict__ g_efield,
                                                     const double* __restrict__ g_efgrad, double* __restrict__ qeff,
                                                     double* __restrict__ facc, double* __restrict__ det) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int j = blockIdx.x * 256 + threadIdx.x;
  const double ge = gE ? gE[0] : 1.0;
  double v[1] = {0.0};
  if (j < fr.nq) {
    const int r = fr.qoff + j;
    double* o = qeff + 10 * (size_t)r;
    o[0] = ge * Q[r] + (g_phi ? g_phi[r] : 0.0);
    for (int t = 0; t < 3; t++) o[1 + t] = ge * mu[3 * (size_t)r + t] - (g_efield ? g_efield[3 * (size_t)r + t] : 0.0);
    const double mult[6] = {2.0, 1.0, 1.0, 2.0, 1.0, 2.0};
    for (int t = 0; t < 6; t++)
      o[4 + t] = ge * theta[6 * (size_t)r + t] - (g_efgrad ? mult[t] * g_efgrad[6 * (size_t)r + t] : 0.0);
    v[0] = o[0];
  }
  double tot[1];
  block_sum256<1>(v, tot);
  if (threadIdx.x == 0) {
    if (det)
      det[(size_t)f * gridDim.x + blockIdx.x] = tot[0];
    else if (blockIdx.x * 256 < fr.nq)
      atomicAdd(&facc[f * FA_COUNT + FA_QTOT_EFF], tot[0]);
  }
}

hipError_t launch_eff_moments(const FrameArg& fa, int max_nq, const double* Q, const double* mu, const double* theta,
                              const double* gE, const double* g_phi, const double* g_efield, const double* g_efgrad,
                              Work& w, hipStream_t s) {
  if (max_nq == 0) return hipSuccess;
  dim3 grid((max_nq + 255) / 256, fa.n_frames);
  hipLaunchKernelGGL(k_eff_moments, grid, dim3(256), 0, s, fa, Q, mu, theta, gE, g_phi, g_efield, g_efgrad, w.qeff,
                     w.facc, w.det_eff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !w.det_eff) return e;
  return launch_det_reduce(fa, 0, 1, w.det_eff, (int)grid.x, 1, det_map({FA_QTOT_EFF}), w.facc, FA_COUNT, s);
}

// MM outputs: sum the reciprocal partials over column chunks, add the real-space part
// and the background term -(pi/(a^2 V)) Q'_tot of dL/dq.
__global__ __launch_bounds__(256) void k_reduce_mm(Grid g, FrameArg fa, int kc_n, int cap_mm,
                                                   const double* __restrict__ mm4, const double* __restrict__ fpart,
                                                   const double* __restrict__ rpart,
                                                   const double* __restrict__ facc, double* __restrict__ g_mm_xyz,
                                                   double* __restrict__ g_mm_q) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= fr.nm) return;
  const int row = fr.moff + i;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int kc = 0; kc < kc_n; kc++) {
    const double* p = fpart + ((size_t)kc * cap_mm + row) * 4;
    s0 += p[0];
    s1 += p[1];
    s2 += p[2];
    s3 += p[3];
  }
  const double q = mm4[(size_t)3 * cap_mm + row];
  const double* rp = rpart + (size_t)row * 4;
  const double V = fr.box[0] * fr.box[1] * fr.box[2];
  g_mm_xyz[3 * (size_t)row + 0] = q * s1 + rp[1];
  g_mm_xyz[3 * (size_t)row + 1] = q * s2 + rp[2];
  g_mm_xyz[3 * (size_t)row + 2] = q * s3 + rp[3];
  if (g_mm_q) g_mm_q[row] = s0 + rp[0] - g.bgw * kPi / (g.alpha * g.alpha * V) * facc[f * FA_COUNT + FA_QTOT_EFF];
}

hipError_t launch_reduce_mm(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm,
                            double* g_mm_xyz, double* g_mm_q, Work& w, hipStream_t s) {
  if (max_nm == 0) return hipSuccess;
  dim3 grid((max_nm + 255) / 256, fa.n_frames);
  hipLaunchKernelGGL(k_reduce_mm, grid, dim3(256), 0, s, g, fa, t.kc, cap_mm, w.mm4, w.fpart, w.rpart, w.facc,
                     g_mm_xyz, g_mm_q);
  return hipGetLastError();
}

// QM outputs of the backward pass.
__global__ __launch_bounds__(256) void k_finalize_bwd(FrameArg fa, const double* __restrict__ site,
                                                      const double* __restrict__ gE, int qmqm,
                                                      const double* __restrict__ qacc, double* __restrict__ g_qm_xyz,
                                                      double* __restrict__ g_Q, double* __restrict__ g_mu,
                                                      double* __restrict__ g_theta) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= fr.nq) return;
  const int r = fr.qoff + j;
  const double ge = gE ? gE[0] : 1.0;
  const double* qa = qacc + (size_t)r * QA_STRIDE;
  const double* st = site + 10 * (size_t)r;
  const double w = qmqm ? 1.0 : 0.0;
  for (int t = 0; t < 3; t++)
    g_qm_xyz[3 * (size_t)r + t] =
        qa[QA_G_QMMM_SR + t] + qa[QA_G_QMMM_LR + t] + ge * w * (qa[QA_G_QQ_LR + t] + qa[QA_G_QQ_SR + t]);
  g_Q[r] = ge * (st[0] + w * (qa[QA_DQ_QQ_LR] + qa[QA_DQ_QQ_SR]));
  for (int t = 0; t < 3; t++)
    g_mu[3 * (size_t)r + t] = ge * (st[1 + t] + w * (qa[QA_DMU_QQ_LR + t] + qa[QA_DMU_QQ_SR + t]));
  const double mult[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};
  for (int t = 0; t < 6; t++)
    g_theta[6 * (size_t)r + t] = ge * mult[t] * (st[4 + t] + w * (qa[QA_DTH_QQ_LR + t] + qa[QA_DTH_QQ_SR + t]));
}

// Fused forward + adjoint epilogue (one launch after both streams join):
// blocks below n_mm_blocks sum the MM gradient data of their atoms; the last
// block of each frame forms phi, field, field gradient and energy of the QM
// sites and, from the same values, the QM gradients for an upstream gradient
// of 1 (gE = 1: the stored context is scaled later).
__global__ __launch_bounds__(256) void k_finish_fused(Grid g, FrameArg fa, int n_mm_blocks, int kc_n, int cap_mm,
                                                      const double* __restrict__ mm4,
                                                      const double* __restrict__ fpart,
                                                      const double* __restrict__ rpart,
                                                      const double* __restrict__ Q, const double* __restrict__ mu,
                                                      const double* __restrict__ theta, int qmqm,
                                                      const double* __restrict__ qacc,
                                                      const double* __restrict__ facc, double* __restrict__ energy,
                                                      double* __restrict__ phi, double* __restrict__ efield,
                                                      double* __restrict__ efgrad, double* __restrict__ site,
                                                      double* __restrict__ g_mm_xyz, double* __restrict__ g_mm_q,
                                                      double* __restrict__ g_qm_xyz, double* __restrict__ g_Q,
                                                      double* __restrict__ g_mu, double* __restrict__ g_theta) {
  const int f = blockIdx.y;
  const FrameDev fr = get_frame(fa, f);
  const double V = fr.box[0] * fr.box[1] * fr.box[2];
  if ((int)blockIdx.x < n_mm_blocks) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= fr.nm) return;
    const int row = fr.moff + i;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int kc = 0; kc < kc_n; kc++) {
      const double* p = fpart + ((size_t)kc * cap_mm + row) * 4;
      s0 += p[0];
      s1 += p[1];
      s2 += p[2];
      s3 += p[3];
    }
    const double q = mm4[(size_t)3 * cap_mm + row];
    const double* rp = rpart + (size_t)row * 4;
    g_mm_xyz[3 * (size_t)row + 0] = q * s1 + rp[1];
    g_mm_xyz[3 * (size_t)row + 1] = q * s2 + rp[2];
    g_mm_xyz[3 * (size_t)row + 2] = q * s3 + rp[3];
    if (g_mm_q) g_mm_q[row] = s0 + rp[0] - g.bgw * kPi / (g.alpha * g.alpha * V) * facc[f * FA_COUNT + FA_QTOT_EFF];
    return;
  }
  const double bg = -g.bgw * kPi / (g.alpha * g.alpha * V) * facc[f * FA_COUNT + FA_QTOT_MM];
  const double w = qmqm ? 1.0 : 0.0;
  const double mult[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};
  double esum = 0.0;
  for (int j = threadIdx.x; j < fr.nq; j += 256) {
    const int r = fr.qoff + j;
    const double* qa = qacc + (size_t)r * QA_STRIDE;
    const double p = qa[QA_PHI_SR] + qa[QA_PHI_LR] + bg;
    double d[3], h[6];
    for (int t = 0; t < 3; t++) d[t] = qa[QA_DPHI_SR + t] + qa[QA_DPHI_LR + t];
    for (int t = 0; t < 6; t++) h[t] = qa[QA_H_SR + t] + qa[QA_H_LR + t];
    if (phi) phi[r] = p;
    if (efield)
      for (int t = 0; t < 3; t++) efield[3 * (size_t)r + t] = -d[t];
    if (efgrad)
      for (int t = 0; t < 6; t++) efgrad[6 * (size_t)r + t] = -2.0 * h[t];
    if (site) {
      double* o = site + 10 * (size_t)r;
      o[0] = p;
      for (int t = 0; t < 3; t++) o[1 + t] = d[t];
      for (int t = 0; t < 6; t++) o[4 + t] = h[t];
    }
    const double* m = mu + 3 * (size_t)r;
    const double* th = theta + 6 * (size_t)r;
    esum += Q[r] * p + m[0] * d[0] + m[1] * d[1] + m[2] * d[2] + th[0] * h[0] + th[3] * h[3] + th[5] * h[5] +
            2.0 * (th[1] * h[1] + th[2] * h[2] + th[4] * h[4]);
    for (int t = 0; t < 3; t++)
      g_qm_xyz[3 * (size_t)r + t] =
          qa[QA_G_QMMM_SR + t] + qa[QA_G_QMMM_LR + t] + w * (qa[QA_G_QQ_LR + t] + qa[QA_G_QQ_SR + t]);
    g_Q[r] = p + w * (qa[QA_DQ_QQ_LR] + qa[QA_DQ_QQ_SR]);
    for (int t = 0; t < 3; t++) g_mu[3 * (size_t)r + t] = d[t] + w * (qa[QA_DMU_QQ_LR + t] + qa[QA_DMU_QQ_SR + t]);
    for (int t = 0; t < 6; t++)
      g_theta[6 * (size_t)r + t] = mult[t] * (h[t] + w * (qa[QA_DTH_QQ_LR + t] + qa[QA_DTH_QQ_SR + t]));
  }
  double v[1] = {esum}, tot[1];
  block_sum256<1>(v, tot);
  if (threadIdx.x == 0) {
    double e = tot[0];
    if (qmqm) e += facc[f * FA_COUNT + FA_E_QQ_LR] + facc[f * FA_COUNT + FA_E_QQ_SR];
    energy[fr.orig] = e;
  }
}

hipError_t launch_finish_fused(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm,
                               const double* Q, const double* mu, const double* theta, int qmqm, double* energy,
                               double* phi, double* efield, double* efgrad, double* site, double* g_mm_xyz,
                               double* g_mm_q, double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta,
                               Work& w, hipStream_t s) {
  const int nb = (max_nm + 255) / 256;
  dim3 grid(nb + 1, fa.n_frames);
  hipLaunchKernelGGL(k_finish_fused, grid, dim3(256), 0, s, g, fa, nb, t.kc, cap_mm, w.mm4, w.fpart, w.rpart, Q, mu,
                     theta, qmqm, w.qacc, w.facc, energy, phi, efield, efgrad, site, g_mm_xyz, g_mm_q, g_qm_xyz, g_Q,
                     g_mu, g_theta);
  return hipGetLastError();
}

// Moments-only update at fixed geometry (self-consistent-field reuse): the MM
// field at each QM site (phi, grad phi, 1/2 grad grad phi, stored by the
// forward call) is contracted with the new moments; the QM-QM image terms
// come from the accumulators of this call.  One block per frame.
__global__ __launch_bounds__(256) void k_finalize_moments(FrameArg fa, const double* __restrict__ Q,
                                                          const double* __restrict__ mu,
                                                          const double* __restrict__ theta, int qmqm,
                                                          const double* __restrict__ site,
                                                          const double* __restrict__ qacc,
                                                          const double* __restrict__ facc, double* __restrict__ energy,
                                                          double* __restrict__ g_Q, double* __restrict__ g_mu,
                                                          double* __restrict__ g_theta) {
  const int f = blockIdx.x;
  const FrameDev fr = get_frame(fa, f);
  const double w = qmqm ? 1.0 : 0.0;
  const double mult[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};
  double esum = 0.0;
  for (int j = threadIdx.x; j < fr.nq; j += 256) {
    const int r = fr.qoff + j;
    const double* qa = qacc + (size_t)r * QA_STRIDE;
    const double* st = site + 10 * (size_t)r;
    const double* m = mu + 3 * (size_t)r;
    const double* th = theta + 6 * (size_t)r;
    esum += Q[r] * st[0] + m[0] * st[1] + m[1] * st[2] + m[2] * st[3] + th[0] * st[4] + th[3] * st[7] +
            th[5] * st[9] + 2.0 * (th[1] * st[5] + th[2] * st[6] + th[4] * st[8]);
    if (g_Q) g_Q[r] = st[0] + w * (qa[QA_DQ_QQ_LR] + qa[QA_DQ_QQ_SR]);
    if (g_mu)
      for (int t = 0; t < 3; t++) g_mu[3 * (size_t)r + t] = st[1 + t] + w * (qa[QA_DMU_QQ_LR + t] + qa[QA_DMU_QQ_SR + t]);
    if (g_theta)
      for (int t = 0; t < 6; t++)
        g_theta[6 * (size_t)r + t] = mult[t] * (st[4 + t] + w * (qa[QA_DTH_QQ_LR + t] + qa[QA_DTH_QQ_SR + t]));
  }
  double v[1] = {esum}, tot[1];
  block_sum256<1>(v, tot);
  if (threadIdx.x == 0) {
    double e = tot[0];
    if (qmqm) e += facc[f * FA_COUNT + FA_E_QQ_LR] + facc[f * FA_COUNT + FA_E_QQ_SR];
    energy[fr.orig] = e;
  }
}

hipError_t launch_finalize_moments(const FrameArg& fa, const double* Q, const double* mu, const double* theta,
                                   int qmqm, const double* site, double* energy, double* g_Q, double* g_mu,
                                   double* g_theta, Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_moments, dim3(fa.n_frames), dim3(256), 0, s, fa, Q, mu, theta, qmqm, site, w.qacc,
                     w.facc, energy, g_Q, g_mu, g_theta);
  return hipGetLastError();
}

hipError_t launch_finalize_bwd(const FrameArg& fa, int max_nq, const double* site, const double* gE, int qmqm,
                               double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta, Work& w, hipStream_t s) {
  if (max_nq == 0) return hipSuccess;
  dim3 grid((max_nq + 255) / 256, fa.n_frames);
  hipLaunchKernelGGL(k_finalize_bwd, grid, dim3(256), 0, s, fa, site, gE, qmqm, w.qacc, g_qm_xyz, g_Q, g_mu, g_theta);
  return hipGetLastError();
}

// gradients for upstream gE from the stored gradients of E
__global__ __launch_bounds__(256) void k_scale_grads(const double* __restrict__ gE, int nq, int nm,
                                                     const double* __restrict__ gq, const double* __restrict__ gQ,
                                                     const double* __restrict__ gmu, const double* __restrict__ gth,
                                                     const double* __restrict__ gm, const double* __restrict__ gmq,
                                                     double* __restrict__ o_q, double* __restrict__ o_Q,
                                                     double* __restrict__ o_mu, double* __restrict__ o_th,
                                                     double* __restrict__ o_m, double* __restrict__ o_mq) {
  const double ge = gE ? gE[0] : 1.0;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < nq) {
    for (int t = 0; t < 3; t++) o_q[3 * i + t] = ge * gq[3 * i + t];
    o_Q[i] = ge * gQ[i];
    for (int t = 0; t < 3; t++) o_mu[3 * i + t] = ge * gmu[3 * i + t];
    for (int t = 0; t < 6; t++) o_th[6 * i + t] = ge * gth[6 * i + t];
  }
  if (i < nm) {
    for (int t = 0; t < 3; t++) o_m[3 * i + t] = ge * gm[3 * i + t];
    if (o_mq) o_mq[i] = ge * gmq[i];
  }
}

hipError_t launch_scale_grads(const double* gE, int nq, int nm, const double* gq, const double* gQ, const double* gmu,
                              const double* gth, const double* gm, const double* gmq, double* o_q, double* o_Q,
                              double* o_mu, double* o_th, double* o_m, double* o_mq, hipStream_t s) {
  const int n = nq > nm ? nq : nm;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_grads, dim3((n + 255) / 256), dim3(256), 0, s, gE, nq, nm, gq, gQ, gmu, gth, gm, gmq, o_q,
                     o_Q, o_mu, o_th, o_m, o_mq);
  return hipGetLastError();
}

hipError_t launch_prep(const Grid& g, const FrameArg& fa, int max_nq, int max_nm, const double* qm_xyz,
                       const double* Q, const double* mu, const double* theta, const double* mm_xyz,
                       const double* mm_q, Work& w, hipStream_t s, int cap_qm, int cap_mm, int mm_tables,
                       int unit_eff, int parts) {
  const int nmax = max_nq > max_nm ? max_nq : max_nm;
  if (nmax > 0 && (parts & PREP_POS)) {
    dim3 grid((nmax + 255) / 256, fa.n_frames);
    hipLaunchKernelGGL(k_prep_pos, grid, dim3(256), 0, s, fa, qm_xyz, Q, mm_xyz, mm_q, mu, theta, w.qm4, cap_qm,
                       w.mm4, cap_mm, w.qacc, w.qeff, unit_eff, w.facc, unit_eff ? w.rpart : (double*)nullptr,
                       w.det_frame);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (w.det_frame) {
      e = launch_det_reduce(fa, 0, 1, w.det_frame, (int)grid.x, 3, det_map({FA_QTOT_MM, FA_QTOT_QM, FA_QTOT_EFF}),
                            w.facc, FA_COUNT, s);
      if (e != hipSuccess) return e;
    }
  }
  if (max_nm > 0 && mm_tables && (parts & PREP_MM_TAB)) {
    launch_tab(g, fa, 0, mm_tables >= 2 ? 1 : 0, max_nm, w.mm4, cap_mm, w.mm_tab, w.mm_ztab, w.mm_xy, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (w.mm_xy32) {
      e = launch_tab32(g, fa, max_nm, cap_mm, w, s);
      if (e != hipSuccess) return e;
    }
  }
  if (max_nq > 0 && (parts & PREP_QM_TAB)) {
    launch_tab(g, fa, 1, 1, max_nq, w.qm4, cap_qm, w.qm_tab, (double*)nullptr, (double2*)nullptr, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mpe
