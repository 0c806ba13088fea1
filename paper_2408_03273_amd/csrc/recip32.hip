// FP32 variant of the two reciprocal-space hot loops (mixed precision).
//
// The phase tables and the folded adjoint weights are rounded to FP32, the
// contractions run on the FP32 matrix cores (v_mfma_f32_16x16x4f32, twice
// the FP64 rate) and the per-block partial sums are handed on in FP64, so
// that every sum over atom chunks and column chunks, and everything after the
// hot loops, stays FP64.  The formulation is that of the FP64 kernels (folded
// +p/-p pairs, separable phases; paper: SI, multipolar Ewald long-range
// terms): only the element type and the accumulator layout differ.  Its error
// against the FP64 results is reported by the tests, not bounded by the
// parity tolerance.
#include <math.h>

#include <algorithm>

#include "ewald_internal.h"

namespace mpe {

#define DEV __device__ __forceinline__

// v_mfma_f32_16x16x4f32: D(16x16) += A(16x4) B(4x16).  A[i][k] sits in lane
// i + 16k, B[k][j] in lane j + 16k, and element r of D in lane l is
// D[4 (l/16) + r][l%16] (rows in groups of four, unlike the FP64 instruction).
typedef float v4f __attribute__((ext_vector_type(4)));

DEV v4f mfma4f(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

DEV int uniform_int32(int v) { return __builtin_amdgcn_readfirstlane(v); }

DEV double uniform_double32(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffu));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

DEV FrameDev frame32(const FrameArg& fa, int f) {
  FrameDev r = fa.frames ? fa.frames[f] : fa.f0;
  for (int a = 0; a < 3; a++) {
    r.box[a] = uniform_double32(r.box[a]);
    r.inv_box[a] = uniform_double32(r.inv_box[a]);
  }
  r.nq = uniform_int32(r.nq);
  r.nm = uniform_int32(r.nm);
  r.qoff = uniform_int32(r.qoff);
  r.moff = uniform_int32(r.moff);
  r.slot_base = uniform_int32(r.slot_base);
  return r;
}

// ------------------------------------------------------------------ FP32 copies of the operands
// MM rows of the compact x/y table and of the real z table (padding included).
__global__ __launch_bounds__(256) void k_tab32(Grid g, FrameArg fa, int cap_mm, const double2* __restrict__ xy,
                                               const double* __restrict__ ztab, float2* __restrict__ xy32,
                                               float* __restrict__ ztab32) {
  const int f = blockIdx.y;
  const FrameDev fr = frame32(fa, f);
  const int per = g.NXY + g.ZKP;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)fr.nm * per) return;
  const int a = (int)(e / per), u = (int)(e - (long)a * per);
  const size_t row = (size_t)fr.moff + a;
  if (u < g.NXY) {
    const double2 v = xy[row * g.NXY + u];
    xy32[row * g.NXY + u] = make_float2((float)v.x, (float)v.y);
  } else {
    const int c = u - g.NXY;
    ztab32[row * g.ZKP + c] = (float)ztab[row * g.ZKP + c];
  }
}

hipError_t launch_tab32(const Grid& g, const FrameArg& fa, int max_nm, int cap_mm, Work& w, hipStream_t s) {
  if (max_nm == 0) return hipSuccess;
  const long n = (long)max_nm * (g.NXY + g.ZKP);
  dim3 grid((unsigned)((n + 255) / 256), fa.n_frames);
  hipLaunchKernelGGL(k_tab32, grid, dim3(256), 0, s, g, fa, cap_mm, w.mm_xy, w.mm_ztab, w.mm_xy32, w.mm_ztab32);
  return hipGetLastError();
}

// folded adjoint weights of every frame (padding entries are zero in both)
__global__ __launch_bounds__(256) void k_wfrag32(size_t n, const double* __restrict__ src, float* __restrict__ dst) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = (float)src[i];
}

hipError_t launch_wfrag32(const Grid& g, const FrameArg& fa, Work& w, hipStream_t s) {
  const size_t n = (size_t)fa.n_frames * g.NG * g.NK2 * 256;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_wfrag32, dim3((unsigned)blocks), dim3(256), 0, s, n, (const double*)w.wfrag, w.wfrag32);
  return hipGetLastError();
}

// ------------------------------------------------------------------ forward: S_MM on FP32 matrix cores
// As the FP64 matrix-core forward: per K step four atoms, A = [Re C; Im C]
// (16 columns x 4 atoms), B = [cos | sin] z table (4 atoms x 16); CT column
// tiles and NT z tiles per wave; the four waves of a block interleave the K
// steps of one atom chunk and are summed through LDS; the block writes its
// partial S(k) in FP64.
template <int CT, int NT>
__global__ __launch_bounds__(256) void k_sfac_mm_mfma32(Grid g, FrameArg fa, int a_chunk, int ngc, int nac,
                                                        int xcd_remap, const double* __restrict__ mm4, int cap_mm,
                                                        const float2* __restrict__ tab,
                                                        const float* __restrict__ ztab,
                                                        double2* __restrict__ spart) {
  static_assert(CT * NT <= 12, "LDS budget of the block reduction");
  constexpr int NACC = CT * NT * 8;  // accumulator floats per lane
  __shared__ float red[2][NACC * 64];
  __shared__ float s0red[4][CT][2][16];
  const int f = blockIdx.z;
  const FrameDev fr = frame32(fa, f);
  int bid = blockIdx.x;
  if (xcd_remap) {
    const int per = (int)gridDim.x / 8;
    if (bid < 8 * per) bid = (bid % 8) * per + bid / 8;
  }
  const int gc = bid % ngc, ac = bid / ngc;
  if (ac >= nac) return;
  const int a0 = ac * a_chunk;
  if (a0 >= fr.nm) return;  // uniform over the block
  const int a1 = min(fr.nm, a0 + a_chunk);
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int32(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  int cx[CT], cy[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    const int col = min((gc * CT + ct) * 16 + li, g.NCOL - 1);
    const int nx = col / g.NY;
    cx[ct] = nx;
    cy[ct] = g.NX + col - nx * g.NY;
  }
  v4f dr[CT][NT], di[CT][NT];
  float s0r[CT], s0i[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    s0r[ct] = s0i[ct] = 0.f;
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
      dr[ct][nt] = v4f{0.f, 0.f, 0.f, 0.f};
      di[ct][nt] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  const double* __restrict__ qv = mm4 + (size_t)3 * cap_mm + fr.moff;
  const float2* __restrict__ tb = tab + (size_t)fr.moff * g.NXY;
  const float* __restrict__ zb = ztab + (size_t)fr.moff * g.ZKP + li;
  for (int a = a0 + 4 * wave; a < a1; a += 16) {
    const int ai = a + lk;
    const bool ok = ai < a1;
    const int ar = ok ? ai : a0;
    const float q = (float)qv[ar] * (ok ? 1.f : 0.f);
    const float2* __restrict__ row = tb + (size_t)ar * g.NXY;
    float bz[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) bz[nt] = zb[(size_t)ar * g.ZKP + nt * 16];
    float2 ex[CT], ey[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      ex[ct] = row[cx[ct]];
      ey[ct] = row[cy[ct]];
    }
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      const float cr = q * (ex[ct].x * ey[ct].x - ex[ct].y * ey[ct].y);
      const float ci = q * (ex[ct].x * ey[ct].y + ex[ct].y * ey[ct].x);
      s0r[ct] += cr;
      s0i[ct] += ci;
#pragma unroll
      for (int nt = 0; nt < NT; nt++) {
        dr[ct][nt] = mfma4f(cr, bz[nt], dr[ct][nt]);
        di[ct][nt] = mfma4f(ci, bz[nt], di[ct][nt]);
      }
    }
  }
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
  auto store = [&](float* dst) {
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
  auto add = [&](const float* src) {
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
  float* T = red[1];  // T[0][c][j] real parts, T[1][c][j] imaginary parts (NACC*64 = 2*NCL*NJ floats)
  if (wave == 0) {
    add(red[0]);
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int nt = 0; nt < NT; nt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int c = ct * 16 + 4 * lk + r, j = nt * 16 + li;
          T[c * NJ + j] = dr[ct][nt][r];
          T[(NCL + c) * NJ + j] = di[ct][nt][r];
        }
  }
  __syncthreads();
  double2* __restrict__ out = spart + (size_t)(fr.slot_base + ac) * g.NZP * g.NCOL;
  for (int e = threadIdx.x; e < NCL * g.NZ; e += 256) {
    const int c = e / g.NZ, iz = e - c * g.NZ;
    const int col = gc * NCL + c;
    if (col >= g.NCOL) break;
    const int nz = iz - g.mz;
    double2 S;
    if (nz == 0) {
      const int ct = c >> 4, cl = c & 15;
      S.x = (((double)s0red[0][ct][0][cl] + (double)s0red[1][ct][0][cl]) + (double)s0red[2][ct][0][cl]) +
            (double)s0red[3][ct][0][cl];
      S.y = (((double)s0red[0][ct][1][cl] + (double)s0red[1][ct][1][cl]) + (double)s0red[2][ct][1][cl]) +
            (double)s0red[3][ct][1][cl];
    } else {
      const int pj = (nz > 0 ? nz : -nz) - 1;
      const double ur = T[c * NJ + pj], ui = T[(NCL + c) * NJ + pj];
      const double vr = T[c * NJ + g.mz + pj], vi = T[(NCL + c) * NJ + g.mz + pj];
      S = nz > 0 ? make_double2(ur - vi, ui + vr) : make_double2(ur + vi, ui - vr);
    }
    out[(size_t)col * g.NZ + iz] = S;
  }
}

hipError_t launch_sfac_mm32(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                            hipStream_t s) {
  Tuning tm = t;
  tm.fwd_mode = 1;
  const int ngc = fwd_col_groups(g, tm);
  const int nac = (max_nm + t.a_chunk - 1) / t.a_chunk;
  if (nac == 0) return hipSuccess;
  dim3 grid(ngc * nac, 1, fa.n_frames);
  const int xcd = (t.fwd_xcd && fa.n_frames == 1) ? 1 : 0;
#define SF(C, N)                                                                                                   \
  if (t.fwd_ct == C && g.NT == N) {                                                                                \
    hipLaunchKernelGGL((k_sfac_mm_mfma32<C, N>), grid, dim3(256), 0, s, g, fa, t.a_chunk, ngc, nac, xcd, w.mm4, \
                       cap_mm, w.mm_xy32, w.mm_ztab32, w.spart);                                                   \
    return hipGetLastError();                                                                                      \
  }
  SF(1, 1) SF(2, 1) SF(4, 1) SF(1, 2) SF(2, 2) SF(4, 2) SF(1, 3) SF(2, 3) SF(4, 3) SF(1, 4) SF(2, 4)
#undef SF
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ adjoint: MM gradients on FP32 matrix cores
// As the FP64 adjoint with the y phases in LDS: A = z table of 16 atoms per
// wave (all K steps in registers), B = folded weights (Re P, Im P, Re Pz,
// Im Pz) from L2, the block's 64 rows of y phases staged in LDS; the
// epilogue multiplies by conj(e^{i kx x} e^{i ky y}) and sums over its
// columns; per-atom results leave in FP64.  Block order as the FP64 kernel:
// atom-tile major, optionally with the blocks of one tile on one XCD.
template <int NK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_force_mm_eyl32(
    Grid g, FrameArg fa, int kc_n, int xcd_remap, int cap_mm, const float2* __restrict__ tab,
    const float* __restrict__ ztab, const float* __restrict__ wfrag, const double2* __restrict__ wk0,
    double* __restrict__ fpart) {
  extern __shared__ float2 eysh32[];  // [64][NY + 1]
  const int f = blockIdx.z;
  const FrameDev fr = frame32(fa, f);
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int32(threadIdx.x >> 6);
  int bid = blockIdx.x;
  if (xcd_remap) {
    const int per = (int)gridDim.x / 8;
    if (bid < 8 * per) bid = (bid % 8) * per + bid / 8;
  }
  const int tile = bid / kc_n, kc = bid - tile * kc_n;
  const int ablk = tile * 64;
  if (ablk >= fr.nm) return;  // uniform over the block
  const int ys = g.NY + 1;
  for (int e = threadIdx.x; e < 64 * g.NY; e += 256) {
    const int a = e / g.NY, c = e - a * g.NY;
    eysh32[a * ys + c] = tab[(size_t)(fr.moff + min(ablk + a, fr.nm - 1)) * g.NXY + g.NX + c];
  }
  __syncthreads();
  const int a0 = ablk + wave * 16;
  if (a0 >= fr.nm) return;  // no barrier after this point
  const int per = (g.NG + kc_n - 1) / kc_n;
  const int gbeg = kc * per, gend = min(g.NG, gbeg + per);
  const int li = lane & 15, lk = lane >> 4;
  float za[NK];
  {
    const int aA = min(a0 + li, fr.nm - 1);
    const float* __restrict__ zr = ztab + (size_t)(fr.moff + aA) * g.ZKP + lk;
#pragma unroll
    for (int st = 0; st < NK; st++) za[st] = zr[4 * st];
  }
  float acc0[4], acc1[4], acc2[4], acc3[4];
  int arow[4], erow[4];
#pragma unroll
  for (int r = 0; r < 4; r++) {
    acc0[r] = acc1[r] = acc2[r] = acc3[r] = 0.f;
    arow[r] = fr.moff + min(a0 + 4 * lk + r, fr.nm - 1);
    erow[r] = (wave * 16 + 4 * lk + r) * ys;
  }
  // this lane's column in group gbeg, then 16 columns further per group; the
  // x phases of the next group are in flight while a group is contracted
  int colp = gbeg * 16 + li;
  float2 exn[4];
  {
    const int nxp = min(colp, g.NCOL - 1) / g.NY;
#pragma unroll
    for (int r = 0; r < 4; r++) exn[r] = tab[(size_t)arow[r] * g.NXY + nxp];
  }
  for (int grp = gbeg; grp < gend; grp++) {
    const int col = colp;
    const bool cok = col < g.NCOL;
    const int colc = cok ? col : g.NCOL - 1;
    const int nx = colc / g.NY, iy = colc - nx * g.NY;
    float2 ex[4];
#pragma unroll
    for (int r = 0; r < 4; r++) ex[r] = exn[r];
    colp += 16;
    {
      const int nxp = min(colp, g.NCOL - 1) / g.NY;
#pragma unroll
      for (int r = 0; r < 4; r++) exn[r] = tab[(size_t)arow[r] * g.NXY + nxp];
    }
    const double2 w0d = wk0[(size_t)f * g.NG * 16 + grp * 16 + li];
    const float w0x = (float)w0d.x, w0y = (float)w0d.y;
    const float* __restrict__ wg = wfrag + ((size_t)f * g.NG + grp) * NK * 256 + lane;
    v4f Pr = v4f{w0x, w0x, w0x, w0x}, Pi = v4f{w0y, w0y, w0y, w0y};
    v4f Zr = v4f{0.f, 0.f, 0.f, 0.f}, Zi = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < NK; st++) {
      const float b0 = wg[st * 256], b1 = wg[st * 256 + 64], b2 = wg[st * 256 + 128], b3 = wg[st * 256 + 192];
      Pr = mfma4f(za[st], b0, Pr);
      Pi = mfma4f(za[st], b1, Pi);
      Zr = mfma4f(za[st], b2, Zr);
      Zi = mfma4f(za[st], b3, Zi);
    }
    if (cok) {
      const float fnx = (float)nx, fny = (float)(iy - g.my);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        // c = e^{-i(kx x + ky y)} = conj(e^{i kx x} e^{i ky y})
        const float2 e = eysh32[erow[r] + iy];
        const float cx = ex[r].x * e.x - ex[r].y * e.y;
        const float cy = -(ex[r].x * e.y + ex[r].y * e.x);
        const float cpi = cx * Pi[r] + cy * Pr[r];
        acc0[r] += cx * Pr[r] - cy * Pi[r];
        acc1[r] += fnx * cpi;
        acc2[r] += fny * cpi;
        acc3[r] += cx * Zi[r] + cy * Zr[r];
      }
    }
  }
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
    const double kx0 = 2.0 * 3.14159265358979323846 * fr.inv_box[0];
    const double ky0 = 2.0 * 3.14159265358979323846 * fr.inv_box[1];
    const double kz0 = 2.0 * 3.14159265358979323846 * fr.inv_box[2];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int a = a0 + 4 * lk + r;
      if (a < fr.nm) {
        double* o = fpart + ((size_t)kc * cap_mm + fr.moff + a) * 4;
        o[0] = (double)acc0[r];
        o[1] = kx0 * (double)acc1[r];
        o[2] = ky0 * (double)acc2[r];
        o[3] = kz0 * (double)acc3[r];
      }
    }
  }
}

hipError_t launch_force_mm32(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                             hipStream_t s) {
  if (max_nm == 0) return hipSuccess;
  dim3 grid(((max_nm + 63) / 64) * t.kc, 1, fa.n_frames);
  const size_t lds = (size_t)64 * (g.NY + 1) * sizeof(float2);
  const int xcd = (t.bwd_xcd && fa.n_frames == 1) ? 1 : 0;
#define FE(N)                                                                                                      \
  case N:                                                                                                          \
    hipLaunchKernelGGL((k_force_mm_eyl32<N>), grid, dim3(256), lds, s, g, fa, t.kc, xcd, cap_mm, w.mm_xy32,       \
                       w.mm_ztab32, w.wfrag32, w.wk0, w.fpart);                                                    \
    break;
  switch (g.NK2) { FE(2) FE(4) FE(6) FE(8) FE(10) FE(12) FE(14) FE(16) default: return hipErrorInvalidValue; }
#undef FE
  return hipGetLastError();
}

}  // namespace mpe
