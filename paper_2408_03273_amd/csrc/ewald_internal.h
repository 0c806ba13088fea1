// Internal layout shared by the host side of the library and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mpe {

// Per-frame description as the kernels see it.
struct FrameDev {
  double box[3];
  double inv_box[3];
  int nq, nm;        // atoms in this frame
  int qoff, moff;    // first packed row of this frame
  int slot_base;     // first partial-sum slot of the forward structure-factor kernel
  int nc[3];         // real-space cells per axis (edge >= rcut); 0 = no cell list
  int cell_base;     // first entry of this frame in the cell arrays
  int orig;          // index of the frame in the caller's list (per-frame outputs)
  int nimg;          // real-space lattice images per direction beyond the minimum image (rc > L/2)
};

// Frames are either one descriptor passed by value (single-frame calls) or
// a device array (batched calls).
struct FrameArg {
  const FrameDev* frames;  // device array or null
  FrameDev f0;             // used when frames == null
  int n_frames;
};

__host__ __device__ inline int kgrid_nx(int mx) { return mx + 1; }
__host__ __device__ inline int kgrid_ny(int my) { return 2 * my + 1; }
__host__ __device__ inline int kgrid_nz(int mz) { return 2 * mz + 1; }

// Static description of the reciprocal grid and real-space parameters
// (identical for every frame of a plan).
struct Grid {
  int mx, my, mz;
  int NX, NY, NZ;   // nx in [0,mx], ny in [-my,my], nz in [-mz,mz]
  int NCOL;         // NX*NY columns (nx,ny)
  int KF;           // NCOL*NZ reciprocal vectors stored per frame (half space + masked rest)
  int Zc;           // nz chunk of the forward kernel
  int NZP;          // nz padded to a multiple of Zc
  int R;            // complex entries per atom in the phase tables: NX + NY + NZP
  int NXY;          // complex entries per atom in the compact x/y table: NX + NY
  int NG;           // 16-column tiles of the matrix-core kernels
  int ZKP;          // real z-phase table row: cos(p kz0 z), p=1..mz, then sin, zero padded to a multiple of 16
  int NT;           // ZKP/16: 16-wide z tiles of the matrix-core forward kernel
  int NK2;          // K steps of 4 of the matrix-core adjoint kernel: 2*ceil(mz/4) (even, zero padded)
  double alpha, rcut;
  double bgw;       // 1: uniform neutralising background terms included, 0: left out
};

// QM accumulator slots (doubles per QM row, zeroed at the start of each call).
enum QmSlot {
  QA_PHI_SR = 0,    // 1
  QA_DPHI_SR = 1,   // 3
  QA_H_SR = 4,      // 6  (1/2 grad grad phi: xx xy xz yy yz zz)
  QA_PHI_LR = 10,
  QA_DPHI_LR = 11,
  QA_H_LR = 14,
  QA_G_QMMM_SR = 20,  // 3  dL/dR of the QM-MM real-space part (effective moments)
  QA_G_QMMM_LR = 23,  // 3
  QA_G_QQ_LR = 26,    // 3
  QA_DQ_QQ_LR = 29,   // 1
  QA_DMU_QQ_LR = 30,  // 3
  QA_DTH_QQ_LR = 33,  // 6 (derivative w.r.t. each distinct full-matrix element)
  QA_G_QQ_SR = 39,    // 3
  QA_DQ_QQ_SR = 42,   // 1 (includes self and background)
  QA_DMU_QQ_SR = 43,  // 3
  QA_DTH_QQ_SR = 46,  // 6
  QA_COUNT = 52,
  QA_STRIDE = 56
};

// Per-frame scalar accumulators.
enum FrameSlot {
  FA_QTOT_MM = 0,
  FA_QTOT_QM = 1,
  FA_E_QMMM_LR = 2,
  FA_E_QQ_LR = 3,
  FA_E_QQ_SR = 4,   // real space + self + background
  FA_QTOT_EFF = 5,  // sum of effective charges (backward)
  FA_COUNT = 8
};

// Device buffers of a plan (all sized for the plan capacities).
struct Work {
  double* mm4;        // [4][cap_mm]  wrapped x,y,z and q
  double* qm4;        // [4][cap_qm]  wrapped x,y,z and Q
  double2* mm_tab;    // [cap_mm][R]  e^{i 2 pi n x/L}: x (n=0..mx), y (-my..my), z (-mz..mz, zero padded)
  double* mm_ztab;    // [cap_mm][ZKP] cos(2 pi p z/Lz), p=1..mz | sin(2 pi p z/Lz), p=1..mz | zeros
  double2* mm_xy;     // [cap_mm][NXY]  x and y parts of mm_tab, compact (matrix-core kernels)
  double2* qm_tab;    // [cap_qm][R]
  double2* sabc;      // [cap_frames][KF][3]  A, B, C of the QM multipoles
  double2* wk;        // [cap_frames][KF]     backward weights (8 pi/V) g(k) S'_QM(k)
  double2* smm;       // [cap_frames][KF]     S_MM for batched calls
  double* kw;         // [cap_frames][KF]     (8 pi/V) e^{-k^2/4a^2}/k^2 on the half space, else 0
  double* wfrag;      // [cap_frames][NG][NK2][4][64] folded adjoint weights in matrix-core B order (zero padded)
  double2* wk0;       // [cap_frames][NG*16]  W at nz = 0 per column (zero for padding columns)
  double2* spart;     // [cap_slots][NZP][NCOL] partial S_MM sums
  double* fpart;      // [cap_kc][cap_mm][4]  partial MM gradient data (phi, dx, dy, dz)
  double* rpart;      // [cap_mm][4]          real-space MM gradient data
  double* qacc;       // [cap_qm][QA_STRIDE]
  double* qeff;       // [cap_qm][10]         effective moments Q', mu', theta'(stored)
  double* site;       // [cap_qm][10]         phi, grad phi, H for batched calls
  double* facc;       // [cap_frames][FA_COUNT]
  double* one;        // a device 1.0
  FrameDev* frames;   // [cap_frames]
  int* cell_cnt;      // [cap_cells]          atoms per cell, then fill counters
  int* cell_start;    // [cap_cells]          first sorted atom of each cell (+ end entry per frame)
  int* cell_atoms;    // [cap_mm]             frame-local MM indices sorted by cell
  int* atom_cell;     // [cap_mm]             cell of each MM atom
  double* region_e;   // [cap_qm]             per-site energies of the region-I / Gaussian terms
  double* region_cen;  // [4]
  double* region_site; // [cap_qm][kRegionSite]
  double4* region_rd;  // [cap_mm]
  double* region_rk;   // [cap_mm]
  int* region_rf;      // [cap_mm]
  double* region_part; // [cap_qm][kRegionMaxChunks][kRegionNV]
  double* oct_part;   // [kMaxOctCandidates][ceil(cap_mm/256)] block partials of the octupole estimate
  // FP32 reciprocal variant only (null otherwise): FP32 copies of the matrix-core operands
  float2* mm_xy32;    // [cap_mm][NXY]
  float* mm_ztab32;   // [cap_mm][ZKP]
  float* wfrag32;     // [cap_frames][NG][NK2][4][64]
  // deterministic mode only (null otherwise): per-block partial sums, added
  // in a fixed order by k_det_reduce instead of floating-point atomics
  double* det_frame;  // [cap_frames][ceil(max(cap_mm, cap_qm) / 256)][3] charge sums of k_prep_pos
  double* det_eff;    // [cap_frames][ceil(cap_qm / 256)]              effective charge sums
  double* det_smm;    // [cap_frames][ceil(KF / 256)][2]                long-range energies
  double* det_proj;   // [cap_qm][kDetPc][26]                          QM-site projection sums
  double* det_real;   // [cap_qm][kDetChunks][13]                      real-space QM-side sums
  double* det_qq;     // [cap_qm]                                       QM-QM site energies
};

// deterministic mode: at most this many projection blocks per QM site and
// real-space MM chunks per QM site
static constexpr int kDetPc = 32;
static constexpr int kDetChunks = 64;

static constexpr int kMaxCellsPerAxis = 16;

// Tunables of the two hot kernels.
struct Tuning {
  int zc;         // VALU forward nz chunk (template instance)
  int a_chunk;    // forward atoms per block
  int kc;         // backward column chunks
  int bwd_ilp;    // backward kernel: 1|2 VALU Horner (atoms per lane), 3|4 matrix cores (16|32 atoms per
                  // wave), 5 matrix cores with separate epilogue waves, 6 matrix cores
                  // with the y phases of the block's atoms in LDS
  int fwd_pf;     // VALU forward kernel prefetches the next atom's factors
  int fwd_target; // forward blocks the atom chunking aims for
  int fwd_mode;   // 0 VALU forward, 1 matrix-core forward
  int fwd_ct;     // matrix-core forward: 16-column tiles per wave
  int fwd_xcd;    // matrix-core forward: XCD-aware block order
  int fwd_units;  // batched calls: partial-sum slots of the forward (its XCD-aware units)
  int bwd_xcd;    // LDS-y adjoint: XCD-aware block order (single-frame calls)
  int fp32r;      // both hot loops on the FP32 matrix cores (mixed-precision variant)
};

// matrix-core kernels are instantiated for mz <= 32
inline bool mfma_fwd_ok(const Grid& g) { return g.NT >= 1 && g.NT <= 4; }
inline bool mfma_bwd_ok(const Grid& g) { return g.NK2 >= 2 && g.NK2 <= 16; }
// the y-phase LDS tile (NY rows of 16 WV + 1 complex entries) must fit in
// 64 KB: 64 atoms per block, or 32 when the 64-atom tile does not fit
inline size_t eyl_lds_bytes(const Grid& g, int wv) { return (size_t)(16 * wv + 1) * g.NY * 16; }
inline bool mfma_bwd_eyl_ok(const Grid& g) { return mfma_bwd_ok(g) && eyl_lds_bytes(g, 2) <= 65536; }
inline int eyl_waves(const Grid& g) { return eyl_lds_bytes(g, 4) <= 65536 ? 4 : 2; }
// Large y grids: only the rows ny >= 0 in LDS (a row ny < 0 is the conjugate
// of row -ny) when the full 64-atom tile would leave fewer than three blocks
// per CU (160 KB of LDS), i.e. fewer waves per SIMD than the registers allow
inline size_t eyl_half_lds_bytes(const Grid& g) { return (size_t)(16 * 4 + 1) * (g.my + 1) * 16; }
inline bool eyl_half_y(const Grid& g) {
  return eyl_lds_bytes(g, 4) * 3 > 160 * 1024 && eyl_half_lds_bytes(g) <= 65536;
}
// the matrix-core hot loops address one frame's x/y phase table with 32-bit
// buffer offsets
// Batched matrix-core forward, one-dimensional grid over the (frame, atom
// chunk) units (= partial-sum slots): the ngc column-group blocks of a unit are
// consecutive on one XCD (workgroups go to the 8 XCDs in turn) and the units
// are dealt to the XCDs in snake order.  Returns false for a block without a
// unit; else the frame index (the last frame whose first slot is <= the unit:
// frames without atoms own no slot and share the next frame's first slot),
// column group and chunk.
__device__ inline bool fwd_unit(const FrameArg& fa, int units, int ngc, int& f, int& gc, int& ac) {
  const int x = blockIdx.x & 7, p = blockIdx.x >> 3;
  const int j = p / ngc;
  gc = p - j * ngc;
  const int u = 8 * j + ((j & 1) ? 7 - x : x);
  if (u >= units) return false;
  int lo = 0, hi = fa.n_frames - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fa.frames[mid].slot_base <= u) lo = mid; else hi = mid - 1;
  }
  f = lo;
  ac = u - fa.frames[lo].slot_base;
  return true;
}

inline bool tab32_ok(const Grid& g, long nm) { return (size_t)nm * g.NXY * 16 < (size_t(1) << 31); }
// the forward tiles per wave are limited by the LDS of the block reduction
// (64 KB of FP64 partial tiles at CT NT = 8; gfx950 gives a block up to 160 KB)
inline bool mfma_fwd_ct_ok(const Grid& g, int ct) { return (ct == 1 || ct == 2 || ct == 4) && ct * g.NT <= 8; }
inline int fwd_col_groups(const Grid& g, const Tuning& t) {
  return t.fwd_mode == 1 ? (g.NG + t.fwd_ct - 1) / t.fwd_ct : ((g.NCOL + 63) / 64) * (g.NZP / g.Zc);
}

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error; all are asynchronous.
hipError_t launch_zero(double* p, size_t n, hipStream_t s);
// destination slots of a fixed-order sum (deterministic mode)
struct DetMap {
  int n;
  int off[32];
};
hipError_t launch_det_reduce(const FrameArg& fa, int mode, int rows, const double* src, int nb, int stride,
                             const DetMap& map, double* dst, int dst_stride, hipStream_t s);
// wrap positions, clear the QM accumulators, sum the charges, build the phase
// tables (mm_tables: 0 none, 1 x/y complex and real z tables, 2 also complex z);
// unit_eff also sets the effective moments for an upstream gradient of 1 and
// zeroes the real-space MM adjoint data (fused forward + adjoint)
// parts: which of the three stages to launch (positions and sums, MM tables, QM tables)
enum { PREP_POS = 1, PREP_MM_TAB = 2, PREP_QM_TAB = 4, PREP_ALL = 7 };
hipError_t launch_prep(const Grid& g, const FrameArg& fa, int max_nq, int max_nm, const double* qm_xyz,
                       const double* Q, const double* mu, const double* theta, const double* mm_xyz,
                       const double* mm_q, Work& w, hipStream_t s, int cap_qm, int cap_mm, int mm_tables,
                       int unit_eff, int parts = PREP_ALL);
hipError_t launch_sfac_qm(const Grid& g, const FrameArg& fa, int max_nq, const double* Q, const double* mu,
                          const double* theta, const double* qeff, const double* gE, int with_w, Work& w,
                          hipStream_t s);
hipError_t launch_sfac_mm(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                          hipStream_t s);
hipError_t launch_sfac_mm_plain(const Grid& g, const FrameArg& fa, int cap_mm, Work& w, hipStream_t s);
hipError_t launch_reduce_smm(const Grid& g, const Tuning& t, const FrameArg& fa, int plain, double2* smm_out,
                             size_t smm_frame_stride, Work& w, hipStream_t s);
// backward: 0 forward sums, 1 adjoint sums, 2 both
hipError_t launch_project_qm(const Grid& g, const FrameArg& fa, int max_nq, int total_nq, const double2* smm,
                             size_t smm_frame_stride, const double* Q, const double* mu, const double* theta,
                             int backward, int qmqm, Work& w, hipStream_t s);
hipError_t launch_force_mm(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                           hipStream_t s);
// backward: 0 forward sums, 1 QM-side adjoint, 2 both; rpart (zeroed, may be
// null) also receives the MM-side adjoint terms: from each pair of the
// QM-side kernel (mm_groups 0), or from the per-atom kernel over mm_groups
// site groups (deterministic plans: one group)
hipError_t launch_real_qm(const Grid& g, const FrameArg& fa, int max_nq, int max_nm, int cap_qm, int cap_mm,
                          int backward, int fp32, Work& w, hipStream_t s, double* rpart = nullptr,
                          int mm_groups = 0);
// MM side of real space per MM atom into w.rpart: one site group writes each
// atom's four values; several groups add to them (rpart zeroed beforehand)
hipError_t launch_real_mm(const Grid& g, const FrameArg& fa, int max_nq, int max_nm, int cap_qm, int cap_mm,
                          int fp32, Work& w, hipStream_t s, int groups = 1);
// cell list (edge >= rcut) of the MM atoms and the real-space kernels that use it
hipError_t launch_cells(const FrameArg& fa, int max_nm, int cap_mm, Work& w, hipStream_t s);
hipError_t launch_real_cells(const Grid& g, const FrameArg& fa, int max_nq, int cap_qm, int cap_mm, int backward,
                             int fp32, Work& w, hipStream_t s);
hipError_t launch_qmqm(const Grid& g, const FrameArg& fa, int max_nq, int cap_qm, const double* Q, const double* mu,
                       const double* theta, Work& w, hipStream_t s);
hipError_t launch_finalize_fwd(const Grid& g, const FrameArg& fa, const double* Q, const double* mu,
                               const double* theta, int qmqm, double* energy, double* phi, double* efield,
                               double* efgrad, double* site_out, Work& w, hipStream_t s);
hipError_t launch_eff_moments(const FrameArg& fa, int max_nq, const double* Q, const double* mu, const double* theta,
                              const double* gE, const double* g_phi, const double* g_efield, const double* g_efgrad,
                              Work& w, hipStream_t s);
hipError_t launch_reduce_mm(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm,
                            double* g_mm_xyz, double* g_mm_q, Work& w, hipStream_t s);
// fused forward + adjoint: MM gradient sums, QM outputs, energy and QM gradients (gE = 1) in one launch
hipError_t launch_finish_fused(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm,
                               const double* Q, const double* mu, const double* theta, int qmqm, double* energy,
                               double* phi, double* efield, double* efgrad, double* site, double* g_mm_xyz,
                               double* g_mm_q, double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta,
                               Work& w, hipStream_t s);
// moments-only update: energy and dE/d(moments) from the stored MM field and this call's QM-QM sums
hipError_t launch_finalize_moments(const FrameArg& fa, const double* Q, const double* mu, const double* theta,
                                   int qmqm, const double* site, double* energy, double* g_Q, double* g_mu,
                                   double* g_theta, Work& w, hipStream_t s);
hipError_t launch_finalize_bwd(const FrameArg& fa, int max_nq, const double* site, const double* gE, int qmqm,
                               double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta, Work& w, hipStream_t s);

hipError_t launch_scale_grads(const double* gE, int nq, int nm, const double* gq, const double* gQ, const double* gmu,
                              const double* gth, const double* gm, const double* gmq, double* o_q, double* o_Q,
                              double* o_mu, double* o_th, double* o_m, double* o_mq, hipStream_t s);
// Region-I / region-II split: inputs of one frame (device pointers, row-major
// as passed by the caller; kappa may be null)
struct RegionArgs {
  int nq, nm;
  const double* qm_xyz;
  const double* Q;
  const double* mu;
  const double* theta;
  const double* mm_xyz;
  const double* mm_q;
  const double* kappa;
  double box[3];
  double inv_box[3];
  double half_min;  // half the smallest box edge
  double r_region, r_gauss;
};
// workspace of one region call (device): centre and QM extent, per-MM-atom
// offsets, exponents and flags, per-(site, chunk) partial sums
static constexpr int kRegionMaxChunks = 32;
static constexpr int kRegionNV = 13;
static constexpr int kRegionSite = 16;
struct RegionWork {
  double* cen;    // [4]
  double* site;   // [cap_qm][kRegionSite]: offset from the centre (3), (effective) Q, mu, theta
  double4* rd;    // [cap_mm]
  double* rk;     // [cap_mm]
  int* rf;        // [cap_mm]
  double* part;   // [cap_qm][kRegionMaxChunks][kRegionNV]
};
// add the region terms to energy / phi / efield / efgrad (any output but energy may be null)
hipError_t launch_region_forward(const RegionArgs& ra, const RegionWork& rw, double* e_site, double* energy,
                                 double* phi, double* efield, double* efgrad, hipStream_t s);
// add the gradients of gE x (region terms) + upstream site gradients to the gradient outputs
hipError_t launch_region_backward(const RegionArgs& ra, const RegionWork& rw, const double* gE, const double* g_phi,
                                  const double* g_efield, const double* g_efgrad, double* g_qm_xyz, double* g_Q,
                                  double* g_mu, double* g_theta, double* g_mm_xyz, double* g_mm_q, hipStream_t s);

// charge-octupole error estimate of region II for candidates r_first + k r_step
static constexpr int kMaxOctCandidates = 256;
struct OctArgs {
  int nq, nm;
  const double* qm_xyz;
  const double* omega;  // (nq,10) xxx,xxy,xxz,xyy,xyz,xzz,yyy,yyz,yzz,zzz
  const double* mm_xyz;
  const double* mm_q;
  double box[3];
  double r_first, r_step, r_outer;
  int n_r;
};
// part: n_r x ceil(nm/256) doubles of workspace; err (n_r) and r_cut (1, may be null) on the device
hipError_t launch_octupole(const OctArgs& oa, double* part, double eps, double* err, double* r_cut, hipStream_t s);

// FP32 reciprocal variant: operand copies and the two hot loops (matrix-core
// forward with the plan's tile choice, adjoint with the y phases in LDS)
hipError_t launch_tab32(const Grid& g, const FrameArg& fa, int max_nm, int cap_mm, Work& w, hipStream_t s);
hipError_t launch_wfrag32(const Grid& g, const FrameArg& fa, Work& w, hipStream_t s);
hipError_t launch_sfac_mm32(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                            hipStream_t s);
hipError_t launch_force_mm32(const Grid& g, const Tuning& t, const FrameArg& fa, int max_nm, int cap_mm, Work& w,
                             hipStream_t s);
inline bool fp32r_ok(const Grid& g) { return mfma_fwd_ok(g) && mfma_bwd_eyl_ok(g); }
// FP32 forward tiles per wave: the block reduction in FP32 takes half the LDS
inline bool fp32r_ct_ok(const Grid& g, int ct) { return (ct == 1 || ct == 2 || ct == 4) && ct * g.NT <= 12; }

// forward kernel instances available for the nz chunk
bool sfac_mm_has_zc(int zc);
int pick_zc(int NZ);

}  // namespace mpe
