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

// Raw buffer loads: a resource holds a wave-uniform base and a byte count
// (loads past it return zero without touching memory); offsets are a per-lane
// byte offset plus a uniform (scalar) byte offset.
DEV __amdgpu_buffer_rsrc_t buf_rsrc32(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
DEV float2 buf_load_f2(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
DEV float4 buf_load_f4(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
DEV float buf_load_f1(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
DEV double buf_load_d1(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
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

// folded adjoint weights of every frame (padding entries are zero in both).
// A 256-entry K step holds the four B fragments k = 0..3 (Re P, Im P, Re Pz,
// Im Pz) of 64 lanes; the FP64 layout pairs them (entry 128 (k >> 1) + 2 lane
// + (k & 1): two 16-byte loads per lane), the FP32 copy is lane-major (entry
// 4 lane + k), so that a lane reads its four values of a K step as one
// 16-byte load.
__global__ __launch_bounds__(256) void k_wfrag32(size_t n, const double* __restrict__ src, float* __restrict__ dst) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const size_t blk = i >> 8;
    const int rem = (int)(i & 255), lane = (rem & 127) >> 1, k = 2 * (rem >> 7) + (rem & 1);
    dst[(blk << 8) + 4 * lane + k] = (float)src[i];
  }
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
                                                        int xcd_remap, int units, const double* __restrict__ mm4,
                                                        int cap_mm,
                                                        const float2* __restrict__ tab,
                                                        const float* __restrict__ ztab,
                                                        double2* __restrict__ spart) {
  static_assert(CT * NT <= 12, "LDS budget of the block reduction");
  constexpr int NACC = CT * NT * 8;  // accumulator floats per lane
  __shared__ float red[2][NACC * 64];
  __shared__ float s0red[4][CT][2][16];
  // block order as the FP64 kernel's: many frames over (frame, atom chunk)
  // units, one frame with the blocks of an atom chunk on one XCD
  int f = blockIdx.z, gc, ac;
  if (units > 0) {
    if (!fwd_unit(fa, units, ngc, f, gc, ac)) return;
  } else {
    int bid = blockIdx.x;
    if (xcd_remap) {
      const int per = (int)gridDim.x / 8;
      if (bid < 8 * per) bid = (bid % 8) * per + bid / 8;
    }
    gc = bid % ngc;
    ac = bid / ngc;
    if (ac >= nac) return;
  }
  const FrameDev fr = frame32(fa, f);
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
  // operands as in the FP64 kernel: buffer loads from resources that end at
  // the chunk's last atom, one offset per lane and a scalar offset per K step,
  // the next step's loads issued before the current one is contracted (two
  // steps unrolled, order pinned with scheduling barriers)
  const int arow = a0 + 4 * wave + lk;
  const __amdgpu_buffer_rsrc_t qr = buf_rsrc32(mm4 + (size_t)3 * cap_mm + fr.moff, (unsigned)a1 * 8u);
  const __amdgpu_buffer_rsrc_t tr = buf_rsrc32(tab + (size_t)fr.moff * g.NXY, (unsigned)a1 * g.NXY * 8u);
  const __amdgpu_buffer_rsrc_t zr = buf_rsrc32(ztab + (size_t)fr.moff * g.ZKP, (unsigned)a1 * g.ZKP * 4u);
  const int qo = arow * 8, zo = (arow * g.ZKP + li) * 4;
  int xo[CT], yo[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    xo[ct] = (arow * g.NXY + cx[ct]) * 8;
    yo[ct] = (arow * g.NXY + cy[ct]) * 8;
  }
  const int ts = 16 * g.NXY * 8, zs = 16 * g.ZKP * 4;  // bytes per K step (16 atoms)
  const int nst = a0 + 4 * wave < a1 ? (a1 - a0 - 4 * wave + 15) / 16 : 0;
  struct Ops {
    double q;
    float2 ex[CT], ey[CT];
    float bz[NT];
  };
  auto fetch = [&](int i, Ops& o) {
    o.q = buf_load_d1(qr, qo, i * 128);
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      o.ex[ct] = buf_load_f2(tr, xo[ct], i * ts);
      o.ey[ct] = buf_load_f2(tr, yo[ct], i * ts);
    }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) o.bz[nt] = buf_load_f1(zr, zo + nt * 64, i * zs);
  };
  auto step = [&](const Ops& o) {
    const float q = (float)o.q;
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      const float pr = fmaf(o.ex[ct].x, o.ey[ct].x, -o.ex[ct].y * o.ey[ct].y);
      const float pi = fmaf(o.ex[ct].x, o.ey[ct].y, o.ex[ct].y * o.ey[ct].x);
      const float cr = q * pr, ci = q * pi;
      s0r[ct] += cr;
      s0i[ct] += ci;
#pragma unroll
      for (int nt = 0; nt < NT; nt++) {
        dr[ct][nt] = mfma4f(cr, o.bz[nt], dr[ct][nt]);
        di[ct][nt] = mfma4f(ci, o.bz[nt], di[ct][nt]);
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
  if (!tab32_ok(g, max_nm)) return hipErrorInvalidValue;  // the API rejects such frames first
  Tuning tm = t;
  tm.fwd_mode = 1;
  const int ngc = fwd_col_groups(g, tm);
  const int nac = (max_nm + t.a_chunk - 1) / t.a_chunk;
  if (nac == 0) return hipSuccess;
  dim3 grid(ngc * nac, 1, fa.n_frames);
  const int xcd = (t.fwd_xcd && fa.n_frames == 1) ? 1 : 0;
  const int units = (t.fwd_xcd && fa.frames && fa.n_frames > 1) ? t.fwd_units : 0;
  if (units > 0) grid = dim3(8 * ngc * ((units + 7) / 8), 1, 1);
#define SF(C, N)                                                                                                   \
  if (t.fwd_ct == C && g.NT == N) {                                                                                \
    hipLaunchKernelGGL((k_sfac_mm_mfma32<C, N>), grid, dim3(256), 0, s, g, fa, t.a_chunk, ngc, nac, xcd, units, \
                       w.mm4, cap_mm, w.mm_xy32, w.mm_ztab32, w.spart);                                            \
    return hipGetLastError();                                                                                      \
  }
  SF(1, 1) SF(2, 1) SF(4, 1) SF(1, 2) SF(2, 2) SF(4, 2) SF(1, 3) SF(2, 3) SF(4, 3) SF(1, 4) SF(2, 4)
#undef SF
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ adjoint: MM gradients on FP32 matrix cores
// As the FP64 adjoint with the y phases in LDS: A = z table of 16 atoms per
// wave (all K steps in registers), B = folded weights (Re P, Im P, Re Pz,
// Im Pz) from L2, the block's 64 rows of y phases staged in LDS (ny-major,
// rows of 66 entries); the epilogue multiplies by conj(e^{i kx x} e^{i ky y})
// and sums over its columns; per-atom results leave in FP64.  The loop is
// organised as the FP64 kernel's: B through a ring of K steps in flight
// across column groups (one 16-byte load per lane and step from the
// lane-major FP32 weights), buffer loads with scalar offsets, no division or
// branch per group, order pinned with scheduling barriers.  Block order:
// atom-tile major, optionally with the blocks of one tile on one XCD.
constexpr int kEyStride32 = 66;  // LDS row of the FP32 adjoint: 64 atoms + 2 (16-byte aligned rows)

template <int NK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_force_mm_eyl32(
    Grid g, FrameArg fa, int kc_n, int xcd_remap, int cap_mm, const float2* __restrict__ tab,
    const float* __restrict__ ztab, const float* __restrict__ wfrag, const double2* __restrict__ wk0,
    double* __restrict__ fpart) {
  extern __shared__ float2 eysh32[];  // [NY][66]
  constexpr int ES = kEyStride32;
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
  for (int e = threadIdx.x; e < 64 * g.NY; e += 256) {
    const int a = e / g.NY, c = e - a * g.NY;
    eysh32[c * ES + a] = tab[(size_t)(fr.moff + min(ablk + a, fr.nm - 1)) * g.NXY + g.NX + c];
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
#pragma unroll
  for (int r = 0; r < 4; r++) acc0[r] = acc1[r] = acc2[r] = acc3[r] = 0.f;
  // x phases: this lane's rows a0 + 4 lk + r (r = 0..3: one row apart)
  const __amdgpu_buffer_rsrc_t xr = buf_rsrc32(tab + (size_t)fr.moff * g.NXY, (unsigned)fr.nm * g.NXY * 8u);
  const int xoff = (a0 + 4 * lk) * g.NXY * 8;
  const int xrow = g.NXY * 8;
  const int erow = wave * 16 + 4 * lk;  // LDS entry of row r = 0 (rows r follow)
  const int q16 = 16 / g.NY, r16 = 16 - q16 * g.NY;
  const double2* __restrict__ w0f = wk0 + (size_t)f * g.NG * 16;
  const float* __restrict__ wff = wfrag + (size_t)f * g.NG * NK * 256;
  constexpr int BD = NK % 3 == 0 ? 3 : (NK % 4 == 0 && NK <= 4) ? 4 : 2;
  static_assert(NK % BD == 0, "ring depth must divide the K steps");
  float4 bq[BD];
  auto wrsrc = [&](int grp) { return buf_rsrc32(wff + (size_t)grp * NK * 256, NK * 256 * 4); };
  int col = gbeg * 16 + li;
  int nx = col / g.NY, iy = col - nx * g.NY;
  {
    const __amdgpu_buffer_rsrc_t w = wrsrc(min(gbeg, g.NG - 1));  // an empty chunk loads and discards
#pragma unroll
    for (int st = 0; st < BD; st++) bq[st] = buf_load_f4(w, lane * 16, st * 1024);
  }
  for (int grp = gbeg; grp < gend; grp++) {
    float2 ex[4];
    {
      const int vo = xoff + min(nx, g.NX - 1) * 8;
#pragma unroll
      for (int r = 0; r < 4; r++) ex[r] = buf_load_f2(xr, vo, r * xrow);
    }
    const __amdgpu_buffer_rsrc_t wn = wrsrc(min(grp + 1, gend - 1));
    const __amdgpu_buffer_rsrc_t wr = wrsrc(grp);
    const double2 w0d = w0f[grp * 16 + li];
    v4f Pr = v4f{0.f, 0.f, 0.f, 0.f}, Pi = Pr, Zr = Pr, Zi = Pr;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < NK; st++) {
      float4& b = bq[st % BD];
      Pr = mfma4f(za[st], b.x, Pr);
      Pi = mfma4f(za[st], b.y, Pi);
      Zr = mfma4f(za[st], b.z, Zr);
      Zi = mfma4f(za[st], b.w, Zi);
      if (st + BD < NK)
        b = buf_load_f4(wr, lane * 16, (st + BD) * 1024);
      else
        b = buf_load_f4(wn, lane * 16, (st + BD - NK) * 1024);
      __builtin_amdgcn_sched_barrier(0);
    }
    // columns past NCOL have zero weights: their terms vanish without a branch
    const float w0x = (float)w0d.x, w0y = (float)w0d.y;
    const float fnx = (float)nx, fny = (float)(iy - g.my);
    const float4* __restrict__ ey = reinterpret_cast<const float4*>(eysh32 + iy * ES + erow);
    const float4 e01 = ey[0], e23 = ey[1];
    const float2 e[4] = {make_float2(e01.x, e01.y), make_float2(e01.z, e01.w), make_float2(e23.x, e23.y),
                         make_float2(e23.z, e23.w)};
#pragma unroll
    for (int r = 0; r < 4; r++) {
      // c = e^{-i(kx x + ky y)} = conj(e^{i kx x} e^{i ky y}) = cr - i s
      const float pr = Pr[r] + w0x, pi = Pi[r] + w0y;
      const float cr = fmaf(ex[r].x, e[r].x, -ex[r].y * e[r].y);
      const float s = fmaf(ex[r].x, e[r].y, ex[r].y * e[r].x);
      const float cpi = fmaf(cr, pi, -s * pr);
      acc0[r] = fmaf(cr, pr, acc0[r]);
      acc0[r] = fmaf(s, pi, acc0[r]);
      acc1[r] = fmaf(fnx, cpi, acc1[r]);
      acc2[r] = fmaf(fny, cpi, acc2[r]);
      acc3[r] = fmaf(cr, Zi[r], acc3[r]);
      acc3[r] = fmaf(-s, Zr[r], acc3[r]);
    }
    iy += r16;
    nx += q16;
    if (iy >= g.NY) {
      iy -= g.NY;
      nx++;
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
  if (!tab32_ok(g, max_nm)) return hipErrorInvalidValue;  // the API rejects such frames first
  const size_t lds = (size_t)kEyStride32 * g.NY * sizeof(float2);
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
