// C ABI of the multipolar Ewald library: plan, validation, workspace, the
// forward / backward / batched launch sequences, HIP-graph replay and the
// tile autotuner.  See include/mpewald.h for the contract of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/mpewald.h"
#include "ewald_internal.h"

namespace mpe {
hipError_t launch_peak_probe(int kind, int blocks, int iters, double* out, hipStream_t s, double* flops);
}

using namespace mpe;

namespace {

thread_local std::string g_last_error;

ewald_status_t fail(ewald_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(EWALD_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kTargetBlocks = 2048;  // blocks the hot kernels aim for (8 per CU)

}  // namespace

struct ewald_plan {
  ewald_params_t p;
  int device;
  Grid g;
  Tuning t;
  Work w;
  int cap_qm, cap_mm, cap_frames, cap_slots, cap_kc, cap_cells;
  std::vector<void*> allocs;
  std::string describe;
  // batched graph state
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // second stream for the adjoint chain that runs beside the forward chain,
  // third for a single frame's all-pairs real space (from the start)
  hipStream_t aux = nullptr, gaux = nullptr, aux2 = nullptr, gaux2 = nullptr;
  int serial = 0;  // run the adjoint chain on the caller's stream (isolated kernel timings)
  int batch_serial = -1;  // batches on one stream: 1 always, 0 never, -1 by the adjoint's weight size
  int batch_target = 16384;  // matrix-core forward of a batch: blocks its atom chunking aims for
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
  hipEvent_t ev_qside = nullptr, ev_mtab = nullptr;  // QM structure factors done; MM tables done
  hipGraphExec_t gexec = nullptr;
  std::vector<unsigned char> gkey;
  std::vector<FrameDev> host_frames;
  // kernel timing (EWALD_PROFILE)
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<std::string, std::pair<long, double>>> prof_acc;
  bool capturing = false;
  // contexts whose stored gradients belong to other moments than the caller's
  // latest ones (an ewald_moments_update call since their forward call):
  // ewald_backward on them runs the full adjoint for the moments it is given
  std::unordered_set<const void*> stale_ctx;
};

namespace {

bool profiling(const ewald_plan* pl) {
  return (pl->p.flags & (EWALD_PROFILE | EWALD_PROFILE_HOT)) && !pl->capturing;
}

// EWALD_PROFILE_HOT brackets only the two reciprocal-space hot loops
bool profiled_launch(const ewald_plan* pl, const char* name) {
  if (!profiling(pl)) return false;
  if (pl->p.flags & EWALD_PROFILE) return true;
  return strncmp(name, "launch_force_mm(", 16) == 0 || strncmp(name, "launch_sfac_mm(", 15) == 0;
}

hipEvent_t pool_event(ewald_plan* pl) {
  if (!pl->ev_pool.empty()) {
    hipEvent_t e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Bracket one launch with events on its own stream.
struct ProfScope {
  ewald_plan* pl;
  hipStream_t s;
  bool on;
  ProfScope(ewald_plan* p, const char* name, hipStream_t st) : pl(p), s(st), on(profiled_launch(p, name)) {
    if (!on) return;
    ewald_plan::ProfRec r{name, pool_event(pl), pool_event(pl)};
    (void)hipEventRecord(r.a, s);
    pl->prof_pending.push_back(r);
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(pl->prof_pending.back().b, s);
  }
};

// images per direction beyond the minimum image that the real-space sums must
// visit: after minimum imaging |d| <= L/2, so |d + nL| < rc needs |n| < rc/L + 1/2
int real_images(const double box[3], double rcut) {
  const double mn = std::min(box[0], std::min(box[1], box[2]));
  return rcut > 0.5 * mn ? (int)std::floor(rcut / mn + 0.5) : 0;
}

// real space visits up to kMaxImages lattice images per direction (rc up to ~3.5 L)
constexpr int kMaxImages = 3;
// region-I sphere and Gaussian pair cutoff: at most this many box lengths
constexpr double kMaxRegionBoxes = 4.0;

ewald_status_t validate_box(const double box[3], double rcut) {
  for (int a = 0; a < 3; a++)
    if (!(box[a] > 0.0) || !std::isfinite(box[a])) return fail(EWALD_ERR_ARG, "box[%d] must be positive", a);
  if (real_images(box, rcut) > kMaxImages) {
    const double mn = std::min(box[0], std::min(box[1], box[2]));
    return fail(EWALD_ERR_CUTOFF, "rcut %.6g needs more than %d lattice images of the smallest box edge %.6g", rcut,
                kMaxImages, mn);
  }
  return EWALD_OK;
}

Grid make_grid(const ewald_params_t& p) {
  Grid g;
  g.mx = p.kmax[0];
  g.my = p.kmax[1];
  g.mz = p.kmax[2];
  g.NX = g.mx + 1;
  g.NY = 2 * g.my + 1;
  g.NZ = 2 * g.mz + 1;
  g.NCOL = g.NX * g.NY;
  g.KF = g.NCOL * g.NZ;
  g.Zc = pick_zc(g.NZ);
  g.NZP = ((g.NZ + g.Zc - 1) / g.Zc) * g.Zc;
  g.R = g.NX + g.NY + g.NZP;
  g.NXY = g.NX + g.NY;
  g.NG = (g.NCOL + 15) / 16;
  g.ZKP = 16 * ((2 * g.mz + 15) / 16);
  g.NT = g.ZKP / 16;
  g.NK2 = 2 * ((g.mz + 3) / 4);
  g.alpha = p.alpha;
  g.rcut = p.rcut;
  g.bgw = (p.flags & EWALD_NO_BACKGROUND) ? 0.0 : 1.0;
  return g;
}

template <typename T>
ewald_status_t alloc(ewald_plan* pl, T** ptr, size_t count) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(EWALD_ERR_OOM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  pl->allocs.push_back(p);
  *ptr = (T*)p;
  return EWALD_OK;
}

int fwd_kblocks(const ewald_plan* pl) { return fwd_col_groups(pl->g, pl->t); }

// smallest forward block count per atom chunk over the kernel variants (sizes the partial-sum slots)
int min_fwd_kblocks(const Grid& g) {
  Tuning t{};
  t.fwd_mode = 0;
  int kb = fwd_col_groups(g, t);
  t.fwd_mode = 1;
  for (int ct : {1, 2, 4})
    if (mfma_fwd_ct_ok(g, ct)) {
      t.fwd_ct = ct;
      kb = std::min(kb, fwd_col_groups(g, t));
    }
  return std::max(kb, 1);
}

// which MM phase tables the selected kernels read
int mm_tables_for(const ewald_plan* pl) { return pl->t.fwd_mode == 0 ? 2 : 1; }


void free_plan(ewald_plan* pl) {
  if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
  if (pl->ev_in) (void)hipEventDestroy(pl->ev_in);
  if (pl->ev_out) (void)hipEventDestroy(pl->ev_out);
  if (pl->gstream) (void)hipStreamDestroy(pl->gstream);
  if (pl->aux) (void)hipStreamDestroy(pl->aux);
  if (pl->gaux) (void)hipStreamDestroy(pl->gaux);
  if (pl->aux2) (void)hipStreamDestroy(pl->aux2);
  if (pl->gaux2) (void)hipStreamDestroy(pl->gaux2);
  if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
  if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
  if (pl->ev_join2) (void)hipEventDestroy(pl->ev_join2);
  if (pl->ev_qside) (void)hipEventDestroy(pl->ev_qside);
  if (pl->ev_mtab) (void)hipEventDestroy(pl->ev_mtab);
  for (auto& r : pl->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pl->ev_pool) (void)hipEventDestroy(e);
  pl->prof_pending.clear();
  pl->ev_pool.clear();
  for (void* p : pl->allocs) (void)hipFree(p);
  pl->allocs.clear();
}

const char* precision_name(int p) {
  switch (p) {
    case EWALD_FP32_REAL: return "fp32-real";
    case EWALD_FP32_RECIP: return "fp32-recip";
    case EWALD_FP32_REAL | EWALD_FP32_RECIP: return "fp32-real+recip";
    default: return "fp64";
  }
}

void set_describe(ewald_plan* pl) {
  char buf[256];
  static const char* bwd[] = {"",           "valu-horner-1", "valu-horner-2", "mfma-fold-16",
                              "mfma-fold-32", "mfma-fold-ws",  "mfma-fold-eyl"};
  char fwd[64];
  if (pl->t.fwd_mode == 1)
    snprintf(fwd, sizeof(fwd), "mfma-fold ct=%d nt=%d xcd=%d", pl->t.fwd_ct, pl->g.NT, pl->t.fwd_xcd);
  else
    snprintf(fwd, sizeof(fwd), "valu zc=%d nzp=%d", pl->g.Zc, pl->g.NZP);
  snprintf(buf, sizeof(buf), "fwd=%s blocks~%d bwd=%s%s kc=%s kgrid=%dx%dx%d precision=%s", fwd, pl->t.fwd_target,
           bwd[pl->t.bwd_ilp], pl->t.bwd_ilp == 6 ? (pl->t.bwd_xcd ? " xcd=1" : " xcd=0") : "",
           pl->t.kc > 0 ? std::to_string(pl->t.kc).c_str() : "auto", pl->g.NX, pl->g.NY, pl->g.NZ,
           precision_name(pl->p.precision));
  pl->describe = buf;
}

FrameDev make_frame(const double box[3], int nq, int nm, int qoff, int moff, int slot_base, double rcut) {
  FrameDev f;
  memset(&f, 0, sizeof(f));
  for (int a = 0; a < 3; a++) {
    f.box[a] = box[a];
    f.inv_box[a] = 1.0 / box[a];
  }
  f.nq = nq;
  f.nm = nm;
  f.qoff = qoff;
  f.moff = moff;
  f.slot_base = slot_base;
  f.nimg = real_images(box, rcut);
  return f;
}

// Cells of edge >= rcut per axis (capped); the cell list is used only when
// every frame has at least 3 cells per axis, else real space runs over all
// pairs.  Returns whether the cell list is used and fills nc/cell_base.
bool assign_cells(const ewald_plan* pl, FrameDev* frames, int n) {
  // (the cell fill orders atoms with atomics: deterministic plans sum over all pairs)
  bool ok = (pl->p.flags & EWALD_CELL_LIST) != 0 && !(pl->p.flags & EWALD_DETERMINISTIC);
  // Building the list costs a few kernel launches; over all pairs, real space
  // costs one distance test per (QM site, MM atom), and its waves evaluate
  // only the pairs within the cutoff (compacted).  Use cells only when that
  // product is large (measured: 38 million tests over the 64 c4 frames run
  // faster over all pairs, 128 million over the 16 c5 replicas over cells),
  // unless MPEWALD_CELLS forces the choice.
  long pairs = 0;
  for (int f = 0; f < n; f++) pairs += (long)frames[f].nq * frames[f].nm;
  int force = -1;
  if (const char* e = getenv("MPEWALD_CELLS")) force = atoi(e) ? 1 : 0;
  if (force == 0 || (force < 0 && pairs < 64000000L)) ok = false;
  for (int f = 0; f < n && ok; f++)
    for (int a = 0; a < 3; a++)
      if ((int)std::floor(frames[f].box[a] / pl->p.rcut) < 3) ok = false;
  int base = 0;
  for (int f = 0; f < n; f++) {
    for (int a = 0; a < 3; a++)
      frames[f].nc[a] = ok ? std::min(kMaxCellsPerAxis, (int)std::floor(frames[f].box[a] / pl->p.rcut)) : 0;
    frames[f].cell_base = base;
    if (ok) base += frames[f].nc[0] * frames[f].nc[1] * frames[f].nc[2] + 1;
  }
  return ok;
}

// How the all-pairs real space gets its MM-side adjoint terms.  With the
// minimum image only, an MM atom meets few QM sites within the cutoff and the
// QM-side kernel adds each pair's terms to the atom's row (returns 0).  When
// the cutoff reaches beyond half a box length (lattice images, rc ~ L), every
// (site, atom) pair has several images within it, and those per-pair adds to
// one row serialise; the per-atom kernel then sums them, over enough site
// groups to give about 2^19 threads (one group in deterministic plans).
int real_mm_groups(const ewald_plan* pl, const FrameDev* frames, int n) {
  bool images = false;
  long atoms = 0;
  int max_nq = 0;
  for (int f = 0; f < n; f++) {
    images = images || frames[f].nimg > 0;
    atoms += frames[f].nm;
    max_nq = std::max(max_nq, frames[f].nq);
  }
  if (!images || atoms == 0) return 0;
  if (pl->p.flags & EWALD_DETERMINISTIC) return 1;
  const long groups = ((1L << 19) + atoms - 1) / atoms;
  return (int)std::max(1L, std::min<long>(groups, std::max(1, max_nq)));
}

// atoms per forward block so that the grid has about kTargetBlocks blocks
// without exceeding the partial-sum slots.
int choose_a_chunk(const ewald_plan* pl, const std::vector<int>& nms) {
  long total = 0;
  for (int n : nms) total += n;
  const long kb = fwd_kblocks(pl);
  long ac;
  if (nms.size() == 1) {
    // one frame: at most fwd_target blocks (so that a target equal to the
    // resident block count gives one full round)
    const long nac = std::max<long>(1, pl->t.fwd_target / kb);
    ac = (total + nac - 1) / nac;
  } else {
    // many frames: more, smaller chunks than one frame would take, so that
    // the XCD-aware order over (frame, chunk) units balances the XCDs
    const long tgt = pl->t.fwd_mode == 1 ? pl->batch_target : pl->t.fwd_target;
    ac = (kb * total + tgt - 1) / tgt;
  }
  ac = ((ac + 63) / 64) * 64;
  if (ac < 64) ac = 64;
  if (pl->t.a_chunk > 0 && nms.size() == 1) ac = pl->t.a_chunk;  // tuned value (single-frame shapes)
  for (;;) {
    long slots = 0;
    for (int n : nms) slots += (n + ac - 1) / ac;
    if (slots <= pl->cap_slots) break;
    ac *= 2;
  }
  return (int)ac;
}

int choose_kc(const ewald_plan* pl, long total_nm) {
  const long per_block = pl->t.bwd_ilp == 4 ? 128L : pl->t.bwd_ilp >= 3 ? 64L : 256L * (pl->t.bwd_ilp == 1 ? 1 : 2);
  const long ablocks = std::max<long>(1, (total_nm + per_block - 1) / per_block);
  long kc = (kTargetBlocks + ablocks - 1) / ablocks;
  if (pl->t.kc > 0) kc = pl->t.kc;
  kc = std::max<long>(1, std::min<long>(kc, pl->cap_kc));
  kc = std::min<long>(kc, pl->g.NCOL);
  return (int)kc;
}

// The matrix-core hot loops address one frame's x/y phase table with 32-bit
// buffer offsets: a frame may hold fewer than 2^31 / (16 (NX + NY)) MM charges
// (1.8 million at |n| <= 24).
ewald_status_t check_frame_mm(const ewald_plan* pl, long n_mm) {
  if (!tab32_ok(pl->g, n_mm))
    return fail(EWALD_ERR_CAPACITY, "a frame of %ld MM charges exceeds the %ld the kernels address at this k grid",
                n_mm, (long)(((size_t(1) << 31) - 1) / ((size_t)pl->g.NXY * 16)));
  return EWALD_OK;
}

// Caller-owned context of one forward call:
//   S_MM(k) | MM potential data at the QM sites (10 per site) |
//   gradients of E for unit upstream gradient: QM (3+1+3+6 per site), MM (3+1 per atom)
struct CtxView {
  double2* smm;
  double* site;
  double* gq;   // [nq][3]
  double* gQ;   // [nq]
  double* gmu;  // [nq][3]
  double* gth;  // [nq][6]
  double* gm;   // [nm][3]
  double* gmq;  // [nm]
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t ctx_bytes(const Grid& g, int nq, int nm) {
  const size_t q = (size_t)std::max(nq, 1), m = (size_t)std::max(nm, 1);
  return align256((size_t)g.KF * sizeof(double2)) + align256(q * 10 * 8) + 4 * align256(q * 6 * 8) +
         2 * align256(m * 3 * 8);
}

CtxView ctx_view(const Grid& g, void* ctx, int nq, int nm) {
  const size_t q = (size_t)std::max(nq, 1), m = (size_t)std::max(nm, 1);
  char* p = (char*)ctx;
  CtxView v;
  v.smm = (double2*)p;
  p += align256((size_t)g.KF * sizeof(double2));
  v.site = (double*)p;
  p += align256(q * 10 * 8);
  v.gq = (double*)p;
  p += align256(q * 6 * 8);
  v.gQ = (double*)p;
  p += align256(q * 6 * 8);
  v.gmu = (double*)p;
  p += align256(q * 6 * 8);
  v.gth = (double*)p;
  p += align256(q * 6 * 8);
  v.gm = (double*)p;
  p += align256(m * 3 * 8);
  v.gmq = (double*)p;
  return v;
}

ewald_status_t check_arrays(int nq, int nm, const void* qm_xyz, const void* Q, const void* mu, const void* theta,
                            const void* mm_xyz, const void* mm_q) {
  if (nq < 0 || nm < 0) return fail(EWALD_ERR_ARG, "negative atom count");
  if (nq > 0 && (!qm_xyz || !Q || !mu || !theta)) return fail(EWALD_ERR_ARG, "null QM input array");
  if (nm > 0 && (!mm_xyz || !mm_q)) return fail(EWALD_ERR_ARG, "null MM input array");
  return EWALD_OK;
}

// ---------------------------------------------------------------- launch sequences
struct Seq {
  ewald_plan* pl;
  hipStream_t s;
  FrameArg fa;
  int max_nq, max_nm, total_nq, total_nm;
  int plain;
  int fp32;
  int qmqm;
  int cells;  // real space over the cell list
  int mm_groups = 0;  // MM side of real space: 0 per pair, else site groups of the per-atom kernel
};

#define LCHK_P(pl_, s_, name, expr)                                                                 \
  do {                                                                                              \
    hipError_t e_;                                                                                  \
    {                                                                                               \
      ProfScope ps_(pl_, name, s_);                                                                 \
      e_ = (expr);                                                                                  \
    }                                                                                               \
    if (e_ != hipSuccess) return fail(EWALD_ERR_HIP, "launch %s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)
#define LCHK(expr) LCHK_P(pl, q.s, #expr, expr)

ewald_status_t seq_begin(const Seq& q, const double* qm_xyz, const double* Q, const double* mu, const double* theta,
                         const double* mm_xyz, const double* mm_q, int mm_tables, int unit_eff,
                         int parts = PREP_ALL) {
  ewald_plan* pl = q.pl;
  if (q.total_nq > q.max_nq)  // packed rows with gaps: clear every QM row (prep clears only the used ones)
    LCHK(launch_zero(pl->w.qacc, (size_t)q.total_nq * QA_STRIDE, q.s));
  LCHK(launch_zero(pl->w.facc, (size_t)q.fa.n_frames * FA_COUNT, q.s));
  LCHK(launch_prep(pl->g, q.fa, q.max_nq, q.max_nm, qm_xyz, Q, mu, theta, mm_xyz, mm_q, pl->w, q.s, pl->cap_qm,
                   pl->cap_mm, mm_tables, unit_eff, parts));
  if (q.cells) {
    LCHK(launch_zero((double*)pl->w.cell_cnt, (size_t)(pl->cap_cells + 1) / 2, q.s));
    LCHK(launch_cells(q.fa, q.max_nm, pl->cap_mm, pl->w, q.s));
  }
  return EWALD_OK;
}

// with_adjoint: the QM-side projection and the all-pairs real-space kernel
// also accumulate the adjoint sums of the effective moments (real space: QM
// and MM side, the latter into the zeroed rpart)
ewald_status_t seq_forward_tail(const Seq& q, const double* Q, const double* mu, const double* theta, double2* smm,
                                size_t smm_stride, double* energy, double* phi, double* efield, double* efgrad,
                                double* site, int with_adjoint = 0, int early = 0, int finalize = 1) {
  ewald_plan* pl = q.pl;
  const int mode = with_adjoint ? 2 : 0;
  LCHK(launch_reduce_smm(pl->g, pl->t, q.fa, q.plain, smm, smm_stride, pl->w, q.s));
  LCHK(launch_project_qm(pl->g, q.fa, q.max_nq, q.total_nq, smm, smm_stride, Q, mu, theta, mode, q.qmqm, pl->w, q.s));
  if (!early) {  // early: real space and QM-QM were launched before the reciprocal work
    if (q.cells)
      LCHK(launch_real_cells(pl->g, q.fa, q.max_nq, pl->cap_qm, pl->cap_mm, 0, q.fp32, pl->w, q.s));
    else
      LCHK(launch_real_qm(pl->g, q.fa, q.max_nq, q.max_nm, pl->cap_qm, pl->cap_mm, mode, q.fp32, pl->w, q.s,
                          with_adjoint ? pl->w.rpart : nullptr, q.mm_groups));
    if (q.qmqm && q.max_nq > 0) LCHK(launch_qmqm(pl->g, q.fa, q.max_nq, pl->cap_qm, Q, mu, theta, pl->w, q.s));
  }
  if (!finalize) return EWALD_OK;
  LCHK(launch_finalize_fwd(pl->g, q.fa, Q, mu, theta, q.qmqm, energy, phi, efield, efgrad, site, pl->w, q.s));
  return EWALD_OK;
}

ewald_status_t fork_to(ewald_plan* pl, hipStream_t from, hipStream_t to) {
  HIPCHK(hipEventRecord(pl->ev_fork, from));
  HIPCHK(hipStreamWaitEvent(to, pl->ev_fork, 0));
  return EWALD_OK;
}

ewald_status_t join_to(ewald_plan* pl, hipStream_t from, hipStream_t to) {
  HIPCHK(hipEventRecord(pl->ev_join, from));
  HIPCHK(hipStreamWaitEvent(to, pl->ev_join, 0));
  return EWALD_OK;
}

// Forward pass and the gradients of E (upstream gradient 1) in one sequence.
// The reciprocal MM adjoint runs on a second stream beside the forward
// structure factor (each hot loop on the matrix cores or the vector units as
// the plan's tiles choose); both need only the phase tables and the QM
// structure factors.
ewald_status_t seq_fwd_bwd(const Seq& q, hipStream_t aux, hipStream_t aux2, const double* qm_xyz, const double* Q, const double* mu,
                           const double* theta, const double* mm_xyz, const double* mm_q, double2* smm,
                           size_t smm_stride, double* energy, double* phi, double* efield, double* efgrad,
                           double* site, double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta,
                           double* g_mm_xyz, double* g_mm_q) {
  ewald_plan* pl = q.pl;
  Work& w = pl->w;
  const Grid& g = pl->g;
  const int tables = mm_tables_for(pl);
  // positions, charge sums, cleared accumulators, unit effective moments
  ewald_status_t st = seq_begin(q, qm_xyz, Q, mu, theta, mm_xyz, mm_q, tables, 1, PREP_POS);
  if (st != EWALD_OK) return st;
  st = fork_to(pl, q.s, aux);
  if (st != EWALD_OK) return st;
  // a single frame's all-pairs real space (forward, QM- and MM-side adjoint
  // in one pass) needs only the staged positions and unit effective moments:
  // on a third stream from here it fills the GPU while the phase tables and
  // QM structure factors are built (the GPU is far from full then), instead
  // of following the adjoint (FP64 vector work inside the hot-loop window
  // delays the matrix-core issue)
  const bool real_early = q.fa.n_frames == 1 && !q.cells;
  if (real_early) {
    Seq qr = q;
    qr.s = aux2;
    const Seq& q_ = qr;
    {
      const Seq& q = q_;
      HIPCHK(hipStreamWaitEvent(q.s, pl->ev_fork, 0));
      LCHK(launch_real_qm(g, q.fa, q.max_nq, q.max_nm, pl->cap_qm, pl->cap_mm, 2, q.fp32, w, q.s, w.rpart,
                          q.mm_groups));
    }
  }
  // many frames: the QM side first on the caller stream, ahead of the MM
  // tables (beside the table pass's blocks the QM structure factors took
  // ~4x their time alone), and both hot loops after both
  const bool qside_first = q.fa.n_frames > 1;
  {
    Seq qa = q;
    qa.s = qside_first ? q.s : aux;
    const Seq& q_ = qa;
    {
      const Seq& q = q_;
      // second stream: the QM phase tables and structure factors (A, B, C,
      // adjoint weights) first, while the forward hot loop has not yet filled
      // the GPU (behind it they were starved and held the adjoint back); the
      // adjoint hot loop follows as soon as the MM tables are ready
      LCHK(launch_prep(g, q.fa, q.max_nq, q.max_nm, qm_xyz, Q, mu, theta, mm_xyz, mm_q, w, q.s, pl->cap_qm,
                       pl->cap_mm, tables, 1, PREP_QM_TAB));
      LCHK(launch_sfac_qm(g, q.fa, q.max_nq, Q, mu, theta, w.qeff, nullptr, 1, w, q.s));
      HIPCHK(hipEventRecord(pl->ev_qside, q.s));
    }
  }
  // caller stream: MM phase tables and, for a single frame, the (small)
  // QM-QM image sums; with many frames the QM-QM sums are a larger grid that
  // would hold the forward back (the adjoint takes the GPU meanwhile), so
  // they go to the second stream, after real space
  const bool qq_first = q.fa.n_frames == 1;
  LCHK(launch_prep(g, q.fa, q.max_nq, q.max_nm, qm_xyz, Q, mu, theta, mm_xyz, mm_q, w, q.s, pl->cap_qm, pl->cap_mm,
                   tables, 1, PREP_MM_TAB));
  HIPCHK(hipEventRecord(pl->ev_mtab, q.s));
  if (qq_first && q.qmqm && q.max_nq > 0) LCHK(launch_qmqm(g, q.fa, q.max_nq, pl->cap_qm, Q, mu, theta, w, q.s));
  // caller stream: the forward hot loop (with many frames after the QM side,
  // whose structure factors the adjoint needs: a forward grid beside them
  // would starve them and the adjoint would start long after the forward)
  LCHK(launch_sfac_mm(g, pl->t, q.fa, q.max_nm, pl->cap_mm, w, q.s));
  {
    Seq qa = q;
    qa.s = aux;
    const Seq& q_ = qa;
    {
      const Seq& q = q_;
      // second stream: the adjoint hot loop, then real space (forward, QM-
      // and MM-side adjoint in one pass), which runs beside the projection on
      // the caller stream and is needed only by the final epilogue
      HIPCHK(hipStreamWaitEvent(q.s, pl->ev_mtab, 0));
      LCHK(launch_force_mm(g, pl->t, q.fa, q.max_nm, pl->cap_mm, w, q.s));
      if (q.cells) {
        LCHK(launch_real_cells(g, q.fa, q.max_nq, pl->cap_qm, pl->cap_mm, 0, q.fp32, w, q.s));
        LCHK(launch_real_cells(g, q.fa, q.max_nq, pl->cap_qm, pl->cap_mm, 1, q.fp32, w, q.s));
      } else if (!real_early) {
        // one pass: QM side per (site, MM chunk) block, the MM-side terms of
        // each pair into rpart (zeroed by prep; in deterministic mode the
        // launcher takes them from the per-atom kernel instead)
        LCHK(launch_real_qm(g, q.fa, q.max_nq, q.max_nm, pl->cap_qm, pl->cap_mm, 2, q.fp32, w, q.s, w.rpart,
                            q.mm_groups));
      }
      if (!qq_first && q.qmqm && q.max_nq > 0)
        LCHK(launch_qmqm(g, q.fa, q.max_nq, pl->cap_qm, Q, mu, theta, w, q.s));
    }
  }
  HIPCHK(hipStreamWaitEvent(q.s, pl->ev_qside, 0));
  // the adjoint sums of the QM-side projection ride along with the forward ones
  st = seq_forward_tail(q, Q, mu, theta, smm, smm_stride, energy, phi, efield, efgrad, site, 1, 1, 0);
  if (st != EWALD_OK) return st;
  st = join_to(pl, aux, q.s);
  if (st != EWALD_OK) return st;
  if (real_early && aux2 != q.s) {
    HIPCHK(hipEventRecord(pl->ev_join2, aux2));
    HIPCHK(hipStreamWaitEvent(q.s, pl->ev_join2, 0));
  }
  LCHK(launch_finish_fused(g, pl->t, q.fa, q.max_nm, pl->cap_mm, Q, mu, theta, q.qmqm, energy, phi, efield, efgrad,
                           site, g_mm_xyz, g_mm_q, g_qm_xyz, g_Q, g_mu, g_theta, w, q.s));
  return EWALD_OK;
}

}  // namespace

extern "C" {

const char* ewald_last_error(void) { return g_last_error.c_str(); }

const char* ewald_version(void) { return "mpewald 0.1 (gfx950)"; }

ewald_status_t ewald_fp64_probe(int kind, int blocks, int iters, double* out, double* flops, void* stream) {
  g_last_error.clear();
  if (kind != 0 && kind != 1) return fail(EWALD_ERR_ARG, "probe kind must be 0 or 1");
  if (blocks < 1 || blocks > 65536 || iters < 1 || iters > 10000000)
    return fail(EWALD_ERR_ARG, "probe blocks must be in 1..65536 and iters in 1..1e7");
  if (!out || !flops) return fail(EWALD_ERR_ARG, "null probe buffer");
  double f = 0.0;
  const hipError_t e = mpe::launch_peak_probe(kind, blocks, iters, out, (hipStream_t)stream, &f);
  if (e != hipSuccess) return fail(EWALD_ERR_HIP, "probe launch: %s", hipGetErrorString(e));
  *flops = f;
  return EWALD_OK;
}

ewald_status_t ewald_setup(const ewald_params_t* params, ewald_plan** plan) {
  g_last_error.clear();
  if (!params || !plan) return fail(EWALD_ERR_ARG, "null params or plan pointer");
  const ewald_params_t& p = *params;
  if (!(p.alpha > 0.0) || !std::isfinite(p.alpha)) return fail(EWALD_ERR_ARG, "alpha must be positive");
  if (!(p.rcut > 0.0) || !std::isfinite(p.rcut)) return fail(EWALD_ERR_ARG, "rcut must be positive");
  for (int a = 0; a < 3; a++)
    if (p.kmax[a] < 1 || p.kmax[a] > 256) return fail(EWALD_ERR_ARG, "kmax[%d] must be in [1,256]", a);
  ewald_status_t st = validate_box(p.box, p.rcut);
  if (st != EWALD_OK) return st;
  if (p.precision < 0 || p.precision > (EWALD_FP32_REAL | EWALD_FP32_RECIP))
    return fail(EWALD_ERR_ARG, "unknown precision %d", p.precision);
  if (p.flags & ~(EWALD_QMQM | EWALD_PLAIN | EWALD_CELL_LIST | EWALD_PROFILE | EWALD_PROFILE_HOT |
                  EWALD_NO_BACKGROUND | EWALD_DETERMINISTIC))
    return fail(EWALD_ERR_ARG, "unknown flags");
  if (p.max_qm < 0 || p.max_mm < 0 || p.max_frames < 1) return fail(EWALD_ERR_ARG, "bad capacities");
  ewald_plan* pl = new ewald_plan();
  pl->p = p;
  if (hipGetDevice(&pl->device) != hipSuccess) {
    delete pl;
    return fail(EWALD_ERR_HIP, "no HIP device");
  }
  pl->g = make_grid(p);
  pl->t.zc = pl->g.Zc;
  pl->t.a_chunk = 0;
  pl->t.kc = 0;
  pl->t.fwd_pf = 0;
  // matrix-core kernels where instantiated (mz <= 32), else the VALU kernels
  pl->t.fwd_mode = mfma_fwd_ok(pl->g) ? 1 : 0;
  pl->t.fwd_ct = mfma_fwd_ct_ok(pl->g, 2) ? 2 : 1;
  pl->t.fwd_xcd = 1;
  pl->t.bwd_xcd = 1;
  pl->t.fwd_target = pl->t.fwd_mode == 1 ? 1024 : 8192;
  pl->t.bwd_ilp = mfma_bwd_eyl_ok(pl->g) ? 6 : mfma_bwd_ok(pl->g) ? 3 : 2;
  // tile overrides for experiments and tests: MPEWALD_BWD = 1|2 (VALU Horner,
  // atoms per lane), 3|4 (matrix cores, 16|32 atoms per wave), 5 (matrix cores
  // with separate epilogue waves) or 6 (matrix cores, y phases in LDS);
  // MPEWALD_SERIAL = 1 runs the adjoint chain on the caller's stream;
  // MPEWALD_BATCH_SERIAL = 0|1 overrides the batches' choice of one stream;
  // MPEWALD_BATCH_TARGET = a batch's forward block count target; MPEWALD_FWD =
  // 0|1 (VALU | matrix cores); MPEWALD_FWD_CT = 1|2|4 (matrix-core column
  // tiles per wave); MPEWALD_FWD_PF = 0|1 (VALU prefetch); MPEWALD_FWD_TARGET =
  // forward block count target; MPEWALD_FWD_XCD, MPEWALD_BWD_XCD = 0|1
  // (XCD-aware block order); MPEWALD_KC = adjoint column chunks (0: automatic)
  if (const char* e = getenv("MPEWALD_BWD")) {
    const int v = atoi(e);
    if ((v >= 1 && v <= 2) || (v >= 3 && v <= 5 && mfma_bwd_ok(pl->g)) || (v == 6 && mfma_bwd_eyl_ok(pl->g)))
      pl->t.bwd_ilp = v;
  }
  if (const char* e = getenv("MPEWALD_FWD")) {
    const int v = atoi(e);
    if (v == 0 || (v == 1 && mfma_fwd_ok(pl->g))) {
      pl->t.fwd_mode = v;
      pl->t.fwd_target = v == 1 ? 1024 : 8192;
    }
  }
  if (const char* e = getenv("MPEWALD_SERIAL")) pl->serial = atoi(e) ? 1 : 0;
  if (const char* e = getenv("MPEWALD_BATCH_SERIAL")) pl->batch_serial = atoi(e) ? 1 : 0;
  if (const char* e = getenv("MPEWALD_BATCH_TARGET")) {
    const int v = atoi(e);
    if (v >= 64 && v <= 65536) pl->batch_target = v;
  }
  if (const char* e = getenv("MPEWALD_FWD_XCD")) pl->t.fwd_xcd = atoi(e) ? 1 : 0;
  if (const char* e = getenv("MPEWALD_BWD_XCD")) pl->t.bwd_xcd = atoi(e) ? 1 : 0;
  if (const char* e = getenv("MPEWALD_KC")) pl->t.kc = std::max(0, atoi(e));
  if (const char* e = getenv("MPEWALD_FWD_CT")) {
    const int v = atoi(e);
    if (mfma_fwd_ct_ok(pl->g, v)) pl->t.fwd_ct = v;
  }
  if (const char* e = getenv("MPEWALD_FWD_PF")) pl->t.fwd_pf = atoi(e) ? 1 : 0;
  if (p.precision & EWALD_FP32_RECIP) {
    // both hot loops on the FP32 matrix cores: matrix-core forward, LDS-y adjoint
    if (!fp32r_ok(pl->g)) {
      delete pl;
      return fail(EWALD_ERR_ARG, "EWALD_FP32_RECIP needs kmax[2] <= 32 and kmax[1] <= 61");
    }
    pl->t.fp32r = 1;
    pl->t.fwd_mode = 1;
    pl->t.bwd_ilp = 6;
    if (!fp32r_ct_ok(pl->g, pl->t.fwd_ct)) pl->t.fwd_ct = 1;
  }
  if (const char* e = getenv("MPEWALD_FWD_TARGET")) {
    const int v = atoi(e);
    if (v >= 64 && v <= 65536) pl->t.fwd_target = v;
  }
  pl->cap_qm = std::max(p.max_qm, 1);
  pl->cap_mm = std::max(p.max_mm, 1);
  pl->cap_frames = p.max_frames;
  pl->cap_cells = pl->cap_frames * (kMaxCellsPerAxis * kMaxCellsPerAxis * kMaxCellsPerAxis + 1);
  pl->cap_slots = std::max(64, 4 * kTargetBlocks / min_fwd_kblocks(pl->g) + 2 * pl->cap_frames);
  pl->cap_kc = (int)std::max<long>(1, std::min<long>(16, (kTargetBlocks * 256L + pl->cap_mm - 1) / pl->cap_mm));
  const Grid& g = pl->g;
  Work& w = pl->w;
  size_t cm = pl->cap_mm, cq = pl->cap_qm, cf = pl->cap_frames;
#define A(ptr, n)                        \
  do {                                   \
    st = alloc(pl, &(ptr), (n));         \
    if (st != EWALD_OK) {                \
      free_plan(pl);                     \
      delete pl;                         \
      return st;                         \
    }                                    \
  } while (0)
  A(w.mm4, 4 * cm);
  A(w.qm4, 4 * cq);
  A(w.mm_tab, cm * g.R);
  A(w.mm_ztab, cm * g.ZKP);
  A(w.mm_xy, cm * g.NXY);
  A(w.qm_tab, cq * g.R);
  A(w.sabc, cf * g.KF * 3);
  A(w.wk, cf * g.KF);
  A(w.smm, cf * g.KF);
  A(w.kw, cf * g.KF);
  A(w.wfrag, cf * (size_t)g.NG * g.NK2 * 256);
  A(w.wk0, cf * (size_t)g.NG * 16);
  A(w.spart, (size_t)pl->cap_slots * g.NZP * g.NCOL);
  A(w.fpart, (size_t)pl->cap_kc * cm * 4);
  A(w.rpart, cm * 4);
  A(w.qacc, cq * QA_STRIDE);
  A(w.qeff, cq * 10);
  A(w.site, cq * 10);
  A(w.facc, cf * FA_COUNT);
  A(w.one, 1);
  A(w.frames, cf);
  A(w.cell_cnt, (size_t)pl->cap_cells + 2);
  A(w.cell_start, (size_t)pl->cap_cells + 2);
  A(w.cell_atoms, cm);
  A(w.atom_cell, cm);
  A(w.region_e, cq);
  A(w.region_cen, 4);
  A(w.region_site, cq * kRegionSite);
  A(w.region_rd, cm);
  A(w.region_rk, cm);
  A(w.region_rf, cm);
  A(w.region_part, cq * kRegionMaxChunks * kRegionNV);
  A(w.oct_part, (size_t)kMaxOctCandidates * ((cm + 255) / 256));
  if (p.flags & EWALD_DETERMINISTIC) {
    const size_t nb_pos = (std::max(cm, cq) + 255) / 256;
    A(w.det_frame, cf * nb_pos * 3);
    A(w.det_eff, cf * ((cq + 255) / 256));
    A(w.det_smm, cf * (((size_t)g.KF + 255) / 256) * 2);
    A(w.det_proj, cq * kDetPc * 26);
    A(w.det_real, cq * kDetChunks * 13);
    A(w.det_qq, cq);
  }
  if (pl->t.fp32r) {
    A(w.mm_xy32, cm * g.NXY);
    A(w.mm_ztab32, cm * g.ZKP);
    A(w.wfrag32, cf * (size_t)g.NG * g.NK2 * 256);
  }
#undef A
  const double one = 1.0;
  // padding entries of the matrix-core operands are never written by the kernels: zero them once
  if (hipMemset(w.wfrag, 0, sizeof(double) * cf * (size_t)g.NG * g.NK2 * 256) != hipSuccess ||
      hipMemset(w.wk0, 0, sizeof(double2) * cf * (size_t)g.NG * 16) != hipSuccess ||
      hipMemset(w.mm_ztab, 0, sizeof(double) * cm * g.ZKP) != hipSuccess ||
      (w.wfrag32 && hipMemset(w.wfrag32, 0, sizeof(float) * cf * (size_t)g.NG * g.NK2 * 256) != hipSuccess) ||
      (w.mm_ztab32 && hipMemset(w.mm_ztab32, 0, sizeof(float) * cm * g.ZKP) != hipSuccess) ||
      hipMemcpy(w.one, &one, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    free_plan(pl);
    delete pl;
    return fail(EWALD_ERR_HIP, "hipMemcpy failed");
  }
  if (hipStreamCreateWithFlags(&pl->aux, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&pl->aux2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&pl->ev_join2, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&pl->ev_qside, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&pl->ev_mtab, hipEventDisableTiming) != hipSuccess) {
    free_plan(pl);
    delete pl;
    return fail(EWALD_ERR_HIP, "stream or event creation failed");
  }
  set_describe(pl);
  *plan = pl;
  return EWALD_OK;
}

ewald_status_t ewald_destroy(ewald_plan* plan) {
  if (!plan) return EWALD_OK;
  free_plan(plan);
  delete plan;
  return EWALD_OK;
}

ewald_status_t ewald_set_box(ewald_plan* plan, const double box[3]) {
  if (!plan || !box) return fail(EWALD_ERR_ARG, "null plan or box");
  ewald_status_t st = validate_box(box, plan->p.rcut);
  if (st != EWALD_OK) return st;
  for (int a = 0; a < 3; a++) plan->p.box[a] = box[a];
  return EWALD_OK;
}

size_t ewald_ctx_bytes(const ewald_plan* plan, int n_qm, int n_mm) {
  (void)n_mm;
  if (!plan) return 0;
  return ctx_bytes(plan->g, n_qm, n_mm);
}

const char* ewald_plan_describe(const ewald_plan* plan) { return plan ? plan->describe.c_str() : ""; }

ewald_status_t ewald_forward(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* Q, const double* mu,
                             const double* theta, int n_mm, const double* mm_xyz, const double* mm_q,
                             double* energy, double* phi, double* efield, double* efgrad, void* ctx, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(EWALD_ERR_ARG, "null plan");
  ewald_status_t st = check_arrays(n_qm, n_mm, qm_xyz, Q, mu, theta, mm_xyz, mm_q);
  if (st != EWALD_OK) return st;
  if (!energy) return fail(EWALD_ERR_ARG, "null energy output");
  if (n_qm > plan->cap_qm || n_mm > plan->cap_mm)
    return fail(EWALD_ERR_CAPACITY, "n_qm=%d n_mm=%d exceed capacity %d/%d", n_qm, n_mm, plan->cap_qm, plan->cap_mm);
  if (check_frame_mm(plan, n_mm) != EWALD_OK) return EWALD_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  Seq q;
  q.pl = plan;
  q.s = s;
  q.plain = (plan->p.flags & EWALD_PLAIN) ? 1 : 0;
  q.fp32 = (plan->p.precision & EWALD_FP32_REAL) != 0;
  q.qmqm = (plan->p.flags & EWALD_QMQM) ? 1 : 0;
  q.max_nq = q.total_nq = n_qm;
  q.max_nm = q.total_nm = n_mm;
  Tuning saved = plan->t;
  plan->t.a_chunk = q.plain ? 1 << 30 : choose_a_chunk(plan, {n_mm});
  q.fa.frames = nullptr;
  q.fa.f0 = make_frame(plan->p.box, n_qm, n_mm, 0, 0, 0, plan->p.rcut);
  q.fa.n_frames = 1;
  q.cells = assign_cells(plan, &q.fa.f0, 1) ? 1 : 0;
  q.mm_groups = real_mm_groups(plan, &q.fa.f0, 1);
  if (ctx) plan->stale_ctx.erase(ctx);
  if (ctx && !q.plain) {
    plan->t.kc = choose_kc(plan, n_mm);
    CtxView cv = ctx_view(plan->g, ctx, n_qm, n_mm);
    st = seq_fwd_bwd(q, plan->serial ? s : plan->aux, plan->serial ? s : plan->aux2, qm_xyz, Q, mu, theta, mm_xyz, mm_q, cv.smm, plan->g.KF, energy, phi, efield,
                     efgrad, cv.site, cv.gq, cv.gQ, cv.gmu, cv.gth, cv.gm, cv.gmq);
    plan->t = saved;
    return st;
  }
  st = seq_begin(q, qm_xyz, Q, mu, theta, mm_xyz, mm_q, q.plain ? 0 : mm_tables_for(plan), 0);
  if (st == EWALD_OK) {
    hipError_t e;
    {
      ProfScope ps(plan, "launch_sfac_qm", s);
      e = launch_sfac_qm(plan->g, q.fa, n_qm, Q, mu, theta, plan->w.qeff, nullptr, 0, plan->w, s);
    }
    if (e != hipSuccess) st = fail(EWALD_ERR_HIP, "sfac_qm launch: %s", hipGetErrorString(e));
  }
  if (st == EWALD_OK) {
    hipError_t e;
    if (q.plain) {
      ProfScope ps(plan, "launch_sfac_mm_plain", s);
      e = launch_sfac_mm_plain(plan->g, q.fa, plan->cap_mm, plan->w, s);
    } else {
      ProfScope ps(plan, "launch_sfac_mm", s);
      e = launch_sfac_mm(plan->g, plan->t, q.fa, n_mm, plan->cap_mm, plan->w, s);
    }
    if (e != hipSuccess) st = fail(EWALD_ERR_HIP, "sfac_mm launch: %s", hipGetErrorString(e));
  }
  if (st == EWALD_OK) {
    CtxView cv{};
    cv.smm = plan->w.smm;
    cv.site = plan->w.site;
    if (ctx) cv = ctx_view(plan->g, ctx, n_qm, n_mm);
    st = seq_forward_tail(q, Q, mu, theta, cv.smm, plan->g.KF, energy, phi, efield, efgrad, cv.site);
  }
  plan->t = saved;
  return st;
}

ewald_status_t ewald_backward(ewald_plan* plan, const void* ctx, int n_qm, const double* qm_xyz, const double* Q,
                              const double* mu, const double* theta, int n_mm, const double* mm_xyz,
                              const double* mm_q, const double* gE, const double* g_phi, const double* g_efield,
                              const double* g_efgrad, double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta,
                              double* g_mm_xyz, double* g_mm_q, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(EWALD_ERR_ARG, "null plan");
  if (!ctx) return fail(EWALD_ERR_ARG, "null ctx: run ewald_forward with a ctx buffer first");
  ewald_status_t st = check_arrays(n_qm, n_mm, qm_xyz, Q, mu, theta, mm_xyz, mm_q);
  if (st != EWALD_OK) return st;
  if (n_qm > 0 && (!g_qm_xyz || !g_Q || !g_mu || !g_theta)) return fail(EWALD_ERR_ARG, "null QM gradient output");
  if (n_mm > 0 && !g_mm_xyz) return fail(EWALD_ERR_ARG, "null MM gradient output");
  if (n_qm > plan->cap_qm || n_mm > plan->cap_mm)
    return fail(EWALD_ERR_CAPACITY, "n_qm=%d n_mm=%d exceed capacity %d/%d", n_qm, n_mm, plan->cap_qm, plan->cap_mm);
  if (check_frame_mm(plan, n_mm) != EWALD_OK) return EWALD_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  Seq q;
  q.pl = plan;
  q.s = s;
  q.plain = 0;
  q.fp32 = (plan->p.precision & EWALD_FP32_REAL) != 0;
  q.qmqm = (plan->p.flags & EWALD_QMQM) ? 1 : 0;
  q.max_nq = q.total_nq = n_qm;
  q.max_nm = q.total_nm = n_mm;
  Tuning saved = plan->t;
  plan->t.kc = choose_kc(plan, n_mm);
  q.fa.frames = nullptr;
  q.fa.f0 = make_frame(plan->p.box, n_qm, n_mm, 0, 0, 0, plan->p.rcut);
  q.fa.n_frames = 1;
  q.cells = assign_cells(plan, &q.fa.f0, 1) ? 1 : 0;
  q.mm_groups = real_mm_groups(plan, &q.fa.f0, 1);
  CtxView cv = ctx_view(plan->g, (void*)ctx, n_qm, n_mm);
  Work& w = plan->w;
  if (!g_phi && !g_efield && !g_efgrad && !(plan->p.flags & EWALD_PLAIN) && !plan->stale_ctx.count(ctx)) {
    // the forward call stored the gradients of E; L = gE E scales them
    hipError_t e;
    {
      ProfScope ps(plan, "launch_scale_grads", s);
      e = launch_scale_grads(gE, n_qm, n_mm, cv.gq, cv.gQ, cv.gmu, cv.gth, cv.gm, cv.gmq, g_qm_xyz, g_Q, g_mu,
                             g_theta, g_mm_xyz, g_mm_q, s);
    }
    plan->t = saved;
    if (e != hipSuccess) return fail(EWALD_ERR_HIP, "scale launch: %s", hipGetErrorString(e));
    return EWALD_OK;
  }
  const Grid& g = plan->g;
#define STEP(expr)                                                                                     \
  do {                                                                                                 \
    hipError_t e_;                                                                                     \
    {                                                                                                  \
      ProfScope ps_(plan, #expr, s);                                                                   \
      e_ = (expr);                                                                                     \
    }                                                                                                  \
    if (e_ != hipSuccess) {                                                                            \
      plan->t = saved;                                                                                 \
      return fail(EWALD_ERR_HIP, "launch %s: %s", #expr, hipGetErrorString(e_));                      \
    }                                                                                                  \
  } while (0)
  // the matrix-core backward kernel reads the MM phase tables in its epilogue
  st = seq_begin(q, qm_xyz, Q, mu, theta, mm_xyz, mm_q, plan->t.bwd_ilp >= 3 ? 1 : 0, 0);
  if (st != EWALD_OK) {
    plan->t = saved;
    return st;
  }
  STEP(launch_eff_moments(q.fa, n_qm, Q, mu, theta, gE, g_phi, g_efield, g_efgrad, w, s));
  STEP(launch_sfac_qm(g, q.fa, n_qm, Q, mu, theta, w.qeff, gE, 1, w, s));
  STEP(launch_force_mm(g, plan->t, q.fa, n_mm, plan->cap_mm, w, s));
  if (q.cells) {
    STEP(launch_zero(w.rpart, (size_t)plan->cap_mm * 4, s));
    STEP(launch_real_cells(g, q.fa, n_qm, plan->cap_qm, plan->cap_mm, 1, q.fp32, w, s));
  } else {
    // several site groups add into rpart from zero; one group writes it
    if (q.mm_groups > 1) STEP(launch_zero(w.rpart, (size_t)plan->cap_mm * 4, s));
    STEP(launch_real_mm(g, q.fa, n_qm, n_mm, plan->cap_qm, plan->cap_mm, q.fp32, w, s, q.mm_groups));
  }
  STEP(launch_reduce_mm(g, plan->t, q.fa, n_mm, plan->cap_mm, g_mm_xyz, g_mm_q, w, s));
  STEP(launch_project_qm(g, q.fa, n_qm, n_qm, cv.smm, g.KF, Q, mu, theta, 1, q.qmqm, w, s));
  if (!q.cells) STEP(launch_real_qm(g, q.fa, n_qm, n_mm, plan->cap_qm, plan->cap_mm, 1, q.fp32, w, s));
  if (q.qmqm && n_qm > 0) STEP(launch_qmqm(g, q.fa, n_qm, plan->cap_qm, Q, mu, theta, w, s));
  STEP(launch_finalize_bwd(q.fa, n_qm, cv.site, gE, q.qmqm, g_qm_xyz, g_Q, g_mu, g_theta, w, s));
#undef STEP
  plan->t = saved;
  return EWALD_OK;
}

}  // extern "C"

namespace {

// Whether a batch runs its forward+backward chain on one stream.  With many
// frames each hot loop fills the GPU by itself, so running them side by side
// gains little; and the matrix-core adjoint reads one frame's folded weights
// from L2 in every block of the frame, which the forward's stream of phase
// rows evicts once the weights pass about half an XCD's 4 MB L2 (measured:
// 64 frames at kmax 20, 1.1 MB of weights, are 1% faster on two streams; 16
// frames at kmax 32, 4.4 MB, 4-5% faster on one, in FP64 and with the FP32
// reciprocal kernels).
bool batch_one_stream(const ewald_plan* pl) {
  if (pl->batch_serial >= 0) return pl->batch_serial != 0;
  if (pl->t.bwd_ilp < 3) return false;
  const size_t weights = (size_t)pl->g.NG * pl->g.NK2 * 256 * sizeof(double);
  return weights > (size_t)2 << 20;
}

ewald_status_t enqueue_batch(ewald_plan* plan, hipStream_t s, int n_frames, int cells, int mm_groups, int max_nq,
                             int max_nm,
                             int total_nq, int total_nm, const double* qm_xyz, const double* Q, const double* mu,
                             const double* theta, const double* mm_xyz, const double* mm_q, int mode, double* energy,
                             double* phi, double* efield, double* efgrad, double* g_qm_xyz, double* g_Q,
                             double* g_mu, double* g_theta, double* g_mm_xyz, double* g_mm_q) {
  ewald_plan* pl = plan;
  Seq q;
  q.pl = plan;
  q.s = s;
  q.plain = 0;
  q.fp32 = (plan->p.precision & EWALD_FP32_REAL) != 0;
  q.qmqm = (plan->p.flags & EWALD_QMQM) ? 1 : 0;
  q.max_nq = max_nq;
  q.max_nm = max_nm;
  q.total_nq = total_nq;
  q.total_nm = total_nm;
  q.fa.frames = plan->w.frames;
  q.fa.n_frames = n_frames;
  memset(&q.fa.f0, 0, sizeof(q.fa.f0));
  q.cells = cells;
  q.mm_groups = mm_groups;
  Work& w = plan->w;
  const Grid& g = plan->g;
  if (mode == EWALD_FWD_BWD) {
    const bool one = plan->serial || batch_one_stream(plan);
    return seq_fwd_bwd(q, one ? s : plan->gaux, one ? s : plan->gaux2, qm_xyz, Q, mu, theta, mm_xyz, mm_q, w.smm,
                       g.KF, energy, phi, efield, efgrad, w.site, g_qm_xyz, g_Q, g_mu, g_theta, g_mm_xyz, g_mm_q);
  }
  ewald_status_t st = seq_begin(q, qm_xyz, Q, mu, theta, mm_xyz, mm_q, mm_tables_for(pl), 0);
  if (st != EWALD_OK) return st;
  LCHK(launch_sfac_qm(g, q.fa, max_nq, Q, mu, theta, w.qeff, nullptr, 0, w, s));
  LCHK(launch_sfac_mm(g, plan->t, q.fa, max_nm, plan->cap_mm, w, s));
  return seq_forward_tail(q, Q, mu, theta, w.smm, g.KF, energy, phi, efield, efgrad, w.site);
}

template <typename T>
void key_push(std::vector<unsigned char>& k, const T& v) {
  const unsigned char* p = (const unsigned char*)&v;
  k.insert(k.end(), p, p + sizeof(T));
}

}  // namespace

extern "C" ewald_status_t ewald_batch(ewald_plan* plan, int n_frames, const ewald_frame_t* frames,
                                      const double* qm_xyz, const double* Q, const double* mu, const double* theta,
                                      const double* mm_xyz, const double* mm_q, int mode, double* energy,
                                      double* phi, double* efield, double* efgrad, double* g_qm_xyz, double* g_Q,
                                      double* g_mu, double* g_theta, double* g_mm_xyz, double* g_mm_q,
                                      void* stream) {
  g_last_error.clear();
  if (!plan || !frames || !energy) return fail(EWALD_ERR_ARG, "null plan, frames or energy");
  if (n_frames < 1) return fail(EWALD_ERR_ARG, "n_frames must be >= 1");
  if (n_frames > plan->cap_frames) return fail(EWALD_ERR_CAPACITY, "%d frames exceed capacity %d", n_frames, plan->cap_frames);
  if (mode != EWALD_FWD && mode != EWALD_FWD_BWD) return fail(EWALD_ERR_ARG, "unknown mode %d", mode);
  int max_nq = 0, max_nm = 0;
  long total_nq = 0, total_nm = 0, end_q = 0, end_m = 0;
  for (int f = 0; f < n_frames; f++) {
    const ewald_frame_t& fr = frames[f];
    ewald_status_t st = validate_box(fr.box, plan->p.rcut);
    if (st != EWALD_OK) return fail(st, "frame %d: %s", f, g_last_error.c_str());
    if (fr.n_qm < 0 || fr.n_mm < 0 || fr.qm_offset < 0 || fr.mm_offset < 0)
      return fail(EWALD_ERR_ARG, "frame %d: negative count or offset", f);
    max_nq = std::max(max_nq, fr.n_qm);
    max_nm = std::max(max_nm, fr.n_mm);
    total_nq += fr.n_qm;
    total_nm += fr.n_mm;
    end_q = std::max(end_q, (long)fr.qm_offset + fr.n_qm);
    end_m = std::max(end_m, (long)fr.mm_offset + fr.n_mm);
  }
  if (end_q > plan->cap_qm || end_m > plan->cap_mm)
    return fail(EWALD_ERR_CAPACITY, "packed rows (%ld QM, %ld MM) exceed capacity %d/%d", end_q, end_m, plan->cap_qm,
                plan->cap_mm);
  if (check_frame_mm(plan, max_nm) != EWALD_OK) return EWALD_ERR_CAPACITY;
  ewald_status_t st = check_arrays((int)total_nq, (int)total_nm, qm_xyz, Q, mu, theta, mm_xyz, mm_q);
  if (st != EWALD_OK) return st;
  if (mode == EWALD_FWD_BWD && ((total_nq > 0 && (!g_qm_xyz || !g_Q || !g_mu || !g_theta)) || (total_nm > 0 && !g_mm_xyz)))
    return fail(EWALD_ERR_ARG, "null gradient output in EWALD_FWD_BWD mode");

  // tile choices for this shape
  std::vector<int> nms(n_frames);
  for (int f = 0; f < n_frames; f++) nms[f] = frames[f].n_mm;
  Tuning saved = plan->t;
  Tuning use = plan->t;
  plan->t.a_chunk = saved.a_chunk;
  use.a_chunk = choose_a_chunk(plan, nms);
  use.kc = choose_kc(plan, total_nm);
  // frame descriptors with partial-sum slots, largest frames first: the grid
  // dimension that runs over frames is dispatched in order, so the longest
  // work starts first and the small frames fill in at the end
  std::vector<int> order(n_frames);
  for (int f = 0; f < n_frames; f++) order[f] = f;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long)frames[a].n_mm * 64 + frames[a].n_qm > (long)frames[b].n_mm * 64 + frames[b].n_qm;
  });
  std::vector<FrameDev> hf(n_frames);
  int slot = 0;
  for (int i = 0; i < n_frames; i++) {
    const ewald_frame_t& fr = frames[order[i]];
    hf[i] = make_frame(fr.box, fr.n_qm, fr.n_mm, fr.qm_offset, fr.mm_offset, slot, plan->p.rcut);
    hf[i].orig = order[i];
    slot += (fr.n_mm + use.a_chunk - 1) / use.a_chunk;
  }
  use.fwd_units = n_frames > 1 ? slot : 0;
  const int cells = assign_cells(plan, hf.data(), n_frames) ? 1 : 0;
  const int mm_groups = real_mm_groups(plan, hf.data(), n_frames);
  // graph key: frames, pointers, mode, stream, tiles
  std::vector<unsigned char> key;
  for (auto& f : hf) key_push(key, f);
  const void* ptrs[] = {qm_xyz, Q, mu, theta, mm_xyz, mm_q, energy, phi, efield, efgrad,
                        g_qm_xyz, g_Q, g_mu, g_theta, g_mm_xyz, g_mm_q, stream};
  for (auto p : ptrs) key_push(key, p);
  key_push(key, mode);
  key_push(key, use);
  hipStream_t s = (hipStream_t)stream;
  if (!plan->gstream) {
    HIPCHK(hipStreamCreateWithFlags(&plan->gstream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&plan->gaux, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&plan->gaux2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&plan->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&plan->ev_out, hipEventDisableTiming));
  }
  if (!plan->gexec || key != plan->gkey) {
    if (plan->gexec) {
      HIPCHK(hipStreamSynchronize(plan->gstream));
      (void)hipGraphExecDestroy(plan->gexec);
      plan->gexec = nullptr;
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(plan->w.frames, hf.data(), sizeof(FrameDev) * n_frames, hipMemcpyHostToDevice));
    plan->t = use;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(plan->gstream, hipStreamCaptureModeThreadLocal));
    plan->capturing = true;
    // QM accumulators are indexed by packed row, so clear every row up to the last one used
    st = enqueue_batch(plan, plan->gstream, n_frames, cells, mm_groups, max_nq, max_nm, (int)end_q, (int)total_nm,
                       qm_xyz, Q, mu, theta, mm_xyz, mm_q, mode, energy, phi, efield, efgrad, g_qm_xyz, g_Q, g_mu,
                       g_theta, g_mm_xyz, g_mm_q);
    hipError_t ce = hipStreamEndCapture(plan->gstream, &graph);
    plan->capturing = false;
    plan->t = saved;
    if (st != EWALD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (ce != hipSuccess) return fail(EWALD_ERR_HIP, "graph capture: %s", hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&plan->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      plan->gexec = nullptr;
      return fail(EWALD_ERR_HIP, "graph instantiate: %s", hipGetErrorString(ie));
    }
    plan->gkey = key;
  }
  HIPCHK(hipEventRecord(plan->ev_in, s));
  HIPCHK(hipStreamWaitEvent(plan->gstream, plan->ev_in, 0));
  HIPCHK(hipGraphLaunch(plan->gexec, plan->gstream));
  HIPCHK(hipEventRecord(plan->ev_out, plan->gstream));
  HIPCHK(hipStreamWaitEvent(s, plan->ev_out, 0));
  return EWALD_OK;
}

// ---------------------------------------------------------------- parameter suggestion
// Truncation tails of the screened sums, relative to the unscreened term at
// the same distance or wave number.  Real space: the order-2 screened tensor
// at r = rcut carries erfc(a r) + (2/sqrt(pi)) a r e^{-a^2 r^2} (1 + 2/3 (a r)^2);
// reciprocal space: the order-2 contraction k.theta.k multiplies the
// Gaussian weight e^{-k^2/4a^2} by (k/2a)^2 relative to the charge term.
namespace {
double real_tail(double a, double rc) {
  const double x = a * rc;
  return std::erfc(x) + 1.1283791670955126 * x * std::exp(-x * x) * (1.0 + 2.0 / 3.0 * x * x);
}
double recip_tail(double a, double k) {
  const double y = k / (2.0 * a);
  return std::exp(-y * y) * (1.0 + y * y);
}
}  // namespace

extern "C" ewald_status_t ewald_suggest_params(const double box[3], double rcut, double tol, double* alpha,
                                               int kmax[3]) {
  g_last_error.clear();
  if (!box || !alpha || !kmax) return fail(EWALD_ERR_ARG, "null argument");
  for (int a = 0; a < 3; a++)
    if (!(box[a] > 0.0) || !std::isfinite(box[a])) return fail(EWALD_ERR_ARG, "box[%d] must be positive", a);
  if (!(rcut > 0.0) || !std::isfinite(rcut)) return fail(EWALD_ERR_ARG, "rcut must be positive");
  if (!(tol > 0.0) || !(tol < 0.1)) return fail(EWALD_ERR_ARG, "tol must be in (0, 0.1)");
  // smallest alpha whose real-space tail at rcut is below tol (the tail falls with alpha)
  double lo = 1e-6 / rcut, hi = 50.0 / rcut;
  if (real_tail(hi, rcut) > tol) return fail(EWALD_ERR_ARG, "tol %.3g below what FP64 real space resolves", tol);
  for (int it = 0; it < 200; it++) {
    const double mid = 0.5 * (lo + hi);
    (real_tail(mid, rcut) > tol ? lo : hi) = mid;
  }
  *alpha = hi;
  // per axis the smallest cube edge whose reciprocal tail at k = 2 pi m / L is below tol
  for (int a = 0; a < 3; a++) {
    int m = 1;
    while (recip_tail(hi, 2.0 * M_PI * m / box[a]) > tol && m < 256) m++;
    if (m >= 256 && recip_tail(hi, 2.0 * M_PI * m / box[a]) > tol)
      return fail(EWALD_ERR_ARG, "box[%d] needs more than 256 reciprocal vectors per direction at tol %.3g", a, tol);
    kmax[a] = m;
  }
  return EWALD_OK;
}

// ---------------------------------------------------------------- moments-only update (SCF reuse)
extern "C" ewald_status_t ewald_moments_update(ewald_plan* plan, const void* ctx, int n_qm, const double* qm_xyz,
                                               const double* Q, const double* mu, const double* theta, int n_mm,
                                               double* energy, double* g_Q, double* g_mu, double* g_theta,
                                               void* stream) {
  g_last_error.clear();
  if (!plan) return fail(EWALD_ERR_ARG, "null plan");
  if (!ctx) return fail(EWALD_ERR_ARG, "null ctx: run ewald_forward with a ctx buffer first");
  if (!energy) return fail(EWALD_ERR_ARG, "null energy output");
  if (n_mm < 0) return fail(EWALD_ERR_ARG, "negative atom count");
  ewald_status_t st = check_arrays(n_qm, 0, qm_xyz, Q, mu, theta, nullptr, nullptr);
  if (st != EWALD_OK) return st;
  if (n_qm > plan->cap_qm || n_mm > plan->cap_mm)
    return fail(EWALD_ERR_CAPACITY, "n_qm=%d n_mm=%d exceed capacity %d/%d", n_qm, n_mm, plan->cap_qm, plan->cap_mm);
  if (check_frame_mm(plan, n_mm) != EWALD_OK) return EWALD_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  // QM-side kernels only: a frame without MM atoms makes S_MM and every QM-MM
  // sum vanish, leaving the QM-QM image terms of the new moments
  Seq q;
  q.pl = plan;
  q.s = s;
  q.plain = 0;
  q.fp32 = 0;
  q.qmqm = (plan->p.flags & EWALD_QMQM) ? 1 : 0;
  q.cells = 0;
  q.max_nq = q.total_nq = n_qm;
  q.max_nm = q.total_nm = 0;
  q.fa.frames = nullptr;
  q.fa.f0 = make_frame(plan->p.box, n_qm, 0, 0, 0, 0, plan->p.rcut);
  q.fa.n_frames = 1;
  const CtxView cv = ctx_view(plan->g, (void*)ctx, n_qm, n_mm);
  Work& w = plan->w;
  const Grid& g = plan->g;
  ewald_plan* pl = plan;
  // the gradients stored in ctx by the forward call are those of its moments
  plan->stale_ctx.insert(ctx);
  st = seq_begin(q, qm_xyz, Q, mu, theta, nullptr, nullptr, 0, 1);
  if (st != EWALD_OK) return st;
  LCHK(launch_sfac_qm(g, q.fa, n_qm, Q, mu, theta, w.qeff, nullptr, 0, w, s));
  if (q.qmqm && n_qm > 0) {
    Tuning tq = plan->t;
    tq.a_chunk = 64;  // no MM atoms: no partial-sum slots to read
    LCHK(launch_reduce_smm(g, tq, q.fa, 0, w.smm, g.KF, w, s));
    LCHK(launch_project_qm(g, q.fa, n_qm, n_qm, w.smm, g.KF, Q, mu, theta, 1, 1, w, s));
    LCHK(launch_qmqm(g, q.fa, n_qm, plan->cap_qm, Q, mu, theta, w, s));
  }
  LCHK(launch_finalize_moments(q.fa, Q, mu, theta, q.qmqm, cv.site, energy, g_Q, g_mu, g_theta, w, s));
  return EWALD_OK;
}

// ---------------------------------------------------------------- region-I / region-II split
static RegionWork region_work(ewald_plan* plan) {
  RegionWork rw;
  rw.cen = plan->w.region_cen;
  rw.site = plan->w.region_site;
  rw.rd = plan->w.region_rd;
  rw.rk = plan->w.region_rk;
  rw.rf = plan->w.region_rf;
  rw.part = plan->w.region_part;
  return rw;
}

static ewald_status_t region_args(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* Q,
                                  const double* mu, const double* theta, int n_mm, const double* mm_xyz,
                                  const double* mm_q, const double* mm_kappa, double r_region, double r_gauss,
                                  RegionArgs& ra) {
  if (!plan) return fail(EWALD_ERR_ARG, "null plan");
  ewald_status_t st = check_arrays(n_qm, n_mm, qm_xyz, Q, mu, theta, mm_xyz, mm_q);
  if (st != EWALD_OK) return st;
  if (n_qm > plan->cap_qm || n_mm > plan->cap_mm)
    return fail(EWALD_ERR_CAPACITY, "n_qm=%d n_mm=%d exceed capacity %d/%d", n_qm, n_mm, plan->cap_qm, plan->cap_mm);
  if (check_frame_mm(plan, n_mm) != EWALD_OK) return EWALD_ERR_CAPACITY;
  if (!std::isfinite(r_region) || !std::isfinite(r_gauss) || r_region < 0.0 || r_gauss < 0.0)
    return fail(EWALD_ERR_ARG, "r_region=%g r_gauss=%g must be finite and >= 0", r_region, r_gauss);
  const double lmin = std::min(plan->p.box[0], std::min(plan->p.box[1], plan->p.box[2]));
  if (r_region > kMaxRegionBoxes * lmin || r_gauss > kMaxRegionBoxes * lmin)
    return fail(EWALD_ERR_CUTOFF, "r_region=%g or r_gauss=%g above %g box lengths (%g)", r_region, r_gauss,
                kMaxRegionBoxes, kMaxRegionBoxes * lmin);
  ra.nq = n_qm;
  ra.nm = n_mm;
  ra.qm_xyz = qm_xyz;
  ra.Q = Q;
  ra.mu = mu;
  ra.theta = theta;
  ra.mm_xyz = mm_xyz;
  ra.mm_q = mm_q;
  ra.kappa = mm_kappa;
  for (int a = 0; a < 3; a++) {
    ra.box[a] = plan->p.box[a];
    ra.inv_box[a] = 1.0 / plan->p.box[a];
  }
  ra.half_min = 0.5 * lmin;
  ra.r_region = r_region;
  ra.r_gauss = r_gauss;
  return EWALD_OK;
}

extern "C" ewald_status_t ewald_region_forward(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* Q,
                                               const double* mu, const double* theta, int n_mm,
                                               const double* mm_xyz, const double* mm_q, const double* mm_kappa,
                                               double r_region, double r_gauss, double* energy, double* phi,
                                               double* efield, double* efgrad, void* stream) {
  g_last_error.clear();
  RegionArgs ra;
  ewald_status_t st = region_args(plan, n_qm, qm_xyz, Q, mu, theta, n_mm, mm_xyz, mm_q, mm_kappa, r_region, r_gauss,
                                  ra);
  if (st != EWALD_OK) return st;
  if (!energy) return fail(EWALD_ERR_ARG, "null energy output");
  ewald_plan* pl = plan;
  hipStream_t s = (hipStream_t)stream;
  LCHK_P(pl, s, "launch_region_forward",
         launch_region_forward(ra, region_work(plan), plan->w.region_e, energy, phi, efield, efgrad, s));
  return EWALD_OK;
}

extern "C" ewald_status_t ewald_region_backward(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* Q,
                                                const double* mu, const double* theta, int n_mm,
                                                const double* mm_xyz, const double* mm_q, const double* mm_kappa,
                                                double r_region, double r_gauss, const double* gE,
                                                const double* g_phi, const double* g_efield,
                                                const double* g_efgrad, double* g_qm_xyz, double* g_Q, double* g_mu,
                                                double* g_theta, double* g_mm_xyz, double* g_mm_q, void* stream) {
  g_last_error.clear();
  RegionArgs ra;
  ewald_status_t st = region_args(plan, n_qm, qm_xyz, Q, mu, theta, n_mm, mm_xyz, mm_q, mm_kappa, r_region, r_gauss,
                                  ra);
  if (st != EWALD_OK) return st;
  if (n_qm > 0 && (!g_qm_xyz || !g_Q || !g_mu || !g_theta)) return fail(EWALD_ERR_ARG, "null QM gradient output");
  if (n_mm > 0 && !g_mm_xyz) return fail(EWALD_ERR_ARG, "null MM gradient output");
  ewald_plan* pl = plan;
  hipStream_t s = (hipStream_t)stream;
  LCHK_P(pl, s, "launch_region_backward",
         launch_region_backward(ra, region_work(plan), gE, g_phi, g_efield, g_efgrad, g_qm_xyz, g_Q, g_mu, g_theta,
                                g_mm_xyz, g_mm_q, s));
  return EWALD_OK;
}

namespace mpe {

ewald_status_t set_error(ewald_status_t st, const char* msg) { return fail(st, "%s", msg); }

void clear_error() { g_last_error.clear(); }

// Host-side checks of the octupole estimate's arguments (shared by the plan
// entry point and its allocation-free variant) and the kernel arguments.
ewald_status_t octupole_args(const double box[3], int n_qm, const double* qm_xyz, const double* omega, int n_mm,
                             const double* mm_xyz, const double* mm_q, int n_r, double r_first, double r_step,
                             double r_outer, double eps, const double* err, OctArgs& oa) {
  if (n_qm < 0 || n_mm < 0) return fail(EWALD_ERR_ARG, "negative atom count");
  if (n_qm > 0 && (!qm_xyz || !omega)) return fail(EWALD_ERR_ARG, "null QM input array");
  if (n_mm > 0 && (!mm_xyz || !mm_q)) return fail(EWALD_ERR_ARG, "null MM input array");
  if (!err) return fail(EWALD_ERR_ARG, "null err output");
  for (int a = 0; a < 3; a++)
    if (!(box[a] > 0.0) || !std::isfinite(box[a])) return fail(EWALD_ERR_ARG, "box[%d] must be positive", a);
  if (n_r < 1 || n_r > kMaxOctCandidates)
    return fail(EWALD_ERR_ARG, "n_r=%d outside [1, %d]", n_r, kMaxOctCandidates);
  const double r_last = r_first + (double)(n_r - 1) * r_step;
  if (!std::isfinite(r_first) || !std::isfinite(r_step) || !std::isfinite(r_last) || !std::isfinite(r_outer) ||
      r_first < 0.0 || r_step < 0.0 || (n_r > 1 && r_step == 0.0) || r_outer < 0.0 || !(eps > 0.0) ||
      !std::isfinite(eps))
    return fail(EWALD_ERR_ARG, "bad candidates r_first=%g r_step=%g r_outer=%g eps=%g", r_first, r_step, r_outer, eps);
  const double lmin = std::min(box[0], std::min(box[1], box[2]));
  if (r_outer > kMaxRegionBoxes * lmin)
    return fail(EWALD_ERR_CUTOFF, "r_outer=%g above %g box lengths (%g)", r_outer, kMaxRegionBoxes,
                kMaxRegionBoxes * lmin);
  oa.nq = n_qm;
  oa.nm = n_mm;
  oa.qm_xyz = qm_xyz;
  oa.omega = omega;
  oa.mm_xyz = mm_xyz;
  oa.mm_q = mm_q;
  for (int a = 0; a < 3; a++) oa.box[a] = box[a];
  oa.r_first = r_first;
  oa.r_step = r_step;
  oa.r_outer = r_outer;
  oa.n_r = n_r;
  return EWALD_OK;
}

}  // namespace mpe

extern "C" ewald_status_t ewald_octupole_error(ewald_plan* plan, int n_qm, const double* qm_xyz,
                                               const double* omega, int n_mm, const double* mm_xyz,
                                               const double* mm_q, int n_r, double r_first, double r_step,
                                               double r_outer, double eps, double* err, double* r_cut,
                                               void* stream) {
  g_last_error.clear();
  if (!plan) return fail(EWALD_ERR_ARG, "null plan");
  if (n_mm > plan->cap_mm) return fail(EWALD_ERR_CAPACITY, "n_mm=%d exceeds capacity %d", n_mm, plan->cap_mm);
  OctArgs oa;
  const ewald_status_t st = octupole_args(plan->p.box, n_qm, qm_xyz, omega, n_mm, mm_xyz, mm_q, n_r, r_first, r_step,
                                          r_outer, eps, err, oa);
  if (st != EWALD_OK) return st;
  ewald_plan* pl = plan;
  hipStream_t s = (hipStream_t)stream;
  LCHK_P(pl, s, "launch_octupole", launch_octupole(oa, plan->w.oct_part, eps, err, r_cut, s));
  return EWALD_OK;
}

// ---------------------------------------------------------------- kernel timing report
extern "C" ewald_status_t ewald_profile_report(ewald_plan* plan, char* buf, size_t len) {
  if (!plan || !buf || len == 0) return fail(EWALD_ERR_ARG, "null plan or buffer");
  for (auto& r : plan->prof_pending) {
    hipError_t e = hipEventSynchronize(r.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return fail(EWALD_ERR_HIP, "profile event: %s", hipGetErrorString(e));
    std::string name(r.name);
    const size_t cut = name.find('(');
    if (cut != std::string::npos) name = name.substr(0, cut);
    if (name.rfind("launch_", 0) == 0) name = name.substr(7);
    bool found = false;
    for (auto& a : plan->prof_acc)
      if (a.first == name) {
        a.second.first += 1;
        a.second.second += ms;
        found = true;
      }
    if (!found) plan->prof_acc.push_back({name, {1, (double)ms}});
    plan->ev_pool.push_back(r.a);
    plan->ev_pool.push_back(r.b);
  }
  plan->prof_pending.clear();
  std::string out = "{";
  for (size_t i = 0; i < plan->prof_acc.size(); i++) {
    char item[160];
    snprintf(item, sizeof(item), "%s\"%s\": {\"count\": %ld, \"total_ms\": %.6f}", i ? ", " : "",
             plan->prof_acc[i].first.c_str(), plan->prof_acc[i].second.first, plan->prof_acc[i].second.second);
    out += item;
  }
  out += "}";
  plan->prof_acc.clear();
  if (out.size() + 1 > len) return fail(EWALD_ERR_ARG, "report needs %zu bytes", out.size() + 1);
  memcpy(buf, out.c_str(), out.size() + 1);
  return EWALD_OK;
}

// ---------------------------------------------------------------- autotuner
namespace {

std::string tune_key(const ewald_plan* pl, int n_mm) {
  int bucket = 1;
  while (bucket < n_mm) bucket <<= 1;
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) arch = prop.gcnArchName;
  const size_t cut = arch.find(':');
  if (cut != std::string::npos) arch = arch.substr(0, cut);
  char buf[160];
  snprintf(buf, sizeof(buf), "%s k%dx%dx%d zc%d nm%d%s", arch.c_str(), pl->g.NX, pl->g.NY, pl->g.NZ, pl->g.Zc, bucket,
           pl->t.fp32r ? " fp32r" : "");
  return buf;
}

bool tune_lookup(ewald_plan* pl, const std::string& key, const char* path) {
  if (!path) return false;
  FILE* fp = fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (fgets(line, sizeof(line), fp)) {
    if (!strstr(line, pat.c_str())) continue;
    int ft = 0, bw = 0, kc = 0, fm = 0, ct = 0;
    const char* p1 = strstr(line, "\"fwd_target\": ");
    const char* p2 = strstr(line, "\"bwd\": ");
    const char* p3 = strstr(line, "\"kc\": ");
    const char* p4 = strstr(line, "\"fwd\": ");
    const char* p5 = strstr(line, "\"ct\": ");
    const char* p6 = strstr(line, "\"xcd\": ");
    const char* p7 = strstr(line, "\"bxcd\": ");
    int xcd = 0, bxcd = 1;
    if (!p6 || sscanf(p6, "\"xcd\": %d", &xcd) != 1) continue;
    if (p7 && sscanf(p7, "\"bxcd\": %d", &bxcd) != 1) continue;
    if (p1 && p2 && p3 && p4 && p5 && sscanf(p1, "\"fwd_target\": %d", &ft) == 1 &&
        sscanf(p2, "\"bwd\": %d", &bw) == 1 && sscanf(p3, "\"kc\": %d", &kc) == 1 &&
        sscanf(p4, "\"fwd\": %d", &fm) == 1 && sscanf(p5, "\"ct\": %d", &ct) == 1 && ft >= 64 &&
        (bw == 1 || bw == 2 || (bw >= 3 && bw <= 5 && mfma_bwd_ok(pl->g)) || (bw == 6 && mfma_bwd_eyl_ok(pl->g))) &&
        kc >= 0 && kc <= pl->cap_kc &&
        (fm == 0 || (fm == 1 && mfma_fwd_ok(pl->g) && mfma_fwd_ct_ok(pl->g, ct)))) {
      pl->t.fwd_target = ft;
      pl->t.bwd_ilp = bw;
      pl->t.kc = kc;
      pl->t.fwd_mode = fm;
      pl->t.fwd_xcd = xcd ? 1 : 0;
      pl->t.bwd_xcd = bxcd ? 1 : 0;
      if (fm == 1) pl->t.fwd_ct = ct;
      found = true;
    }
  }
  fclose(fp);
  return found;
}

}  // namespace

extern "C" ewald_status_t ewald_autotune(ewald_plan* plan, int n_mm, const char* cache_path) {
  g_last_error.clear();
  if (!plan) return fail(EWALD_ERR_ARG, "null plan");
  if (n_mm < 1 || n_mm > plan->cap_mm) return fail(EWALD_ERR_CAPACITY, "n_mm=%d outside 1..%d", n_mm, plan->cap_mm);
  if (check_frame_mm(plan, n_mm) != EWALD_OK) return EWALD_ERR_CAPACITY;
  const std::string key = tune_key(plan, n_mm);
  if (tune_lookup(plan, key, cache_path)) {
    set_describe(plan);
    return EWALD_OK;
  }
  // synthetic frame: uniform MM charges (neutral) and QM multipoles near the
  // centre, as many as the plan holds (up to 64: the QM-side kernels share the
  // GPU with the hot loops in the fused step)
  const int nq = std::min(64, plan->cap_qm);
  std::vector<double> hm(3 * (size_t)n_mm), hq(n_mm), hqp(3 * (size_t)nq), hQ(nq), hmu(3 * (size_t)nq),
      hth(6 * (size_t)nq);
  unsigned long long st64 = 0x9E3779B97F4A7C15ull;
  auto rnd = [&]() {
    st64 = st64 * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(st64 >> 11) * (1.0 / 9007199254740992.0);
  };
  double qs = 0.0;
  for (int i = 0; i < n_mm; i++) {
    for (int a = 0; a < 3; a++) hm[3 * (size_t)i + a] = rnd() * plan->p.box[a];
    hq[i] = rnd() * 1.8 - 0.9;
    qs += hq[i];
  }
  for (int i = 0; i < n_mm; i++) hq[i] -= qs / n_mm;
  for (int j = 0; j < nq; j++) {
    for (int a = 0; a < 3; a++) hqp[3 * j + a] = plan->p.box[a] * (0.45 + 0.1 * rnd());
    hQ[j] = rnd() - 0.5;
    for (int a = 0; a < 3; a++) hmu[3 * j + a] = 0.2 * (rnd() - 0.5);
    for (int a = 0; a < 6; a++) hth[6 * j + a] = 0.1 * (rnd() - 0.5);
  }
  double *dm = nullptr, *dq = nullptr, *dqp = nullptr, *dQ = nullptr, *dmu = nullptr, *dth = nullptr;
  double *d_out = nullptr;  // energy, phi, efield, efgrad of the in-context steps
  void* d_ctx = nullptr;
  std::vector<std::pair<double, Tuning>> fres, bres;  // standalone times of the candidates
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ewald_status_t st = EWALD_OK;
  const Tuning saved = plan->t;
  double best_f = 1e30, best_b = 1e30;
  Tuning best = saved;
  std::string report;
#define TCHK(expr)                                                                  \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      st = fail(EWALD_ERR_HIP, "autotune %s: %s", #expr, hipGetErrorString(e_));    \
      goto done;                                                                    \
    }                                                                               \
  } while (0)
  {
    TCHK(hipMalloc(&dm, hm.size() * 8));
    TCHK(hipMalloc(&dq, hq.size() * 8));
    TCHK(hipMalloc(&dqp, hqp.size() * 8));
    TCHK(hipMalloc(&dQ, hQ.size() * 8));
    TCHK(hipMalloc(&dmu, hmu.size() * 8));
    TCHK(hipMalloc(&dth, hth.size() * 8));
    TCHK(hipMemcpy(dm, hm.data(), hm.size() * 8, hipMemcpyHostToDevice));
    TCHK(hipMemcpy(dq, hq.data(), hq.size() * 8, hipMemcpyHostToDevice));
    TCHK(hipMemcpy(dqp, hqp.data(), hqp.size() * 8, hipMemcpyHostToDevice));
    TCHK(hipMemcpy(dQ, hQ.data(), hQ.size() * 8, hipMemcpyHostToDevice));
    TCHK(hipMemcpy(dmu, hmu.data(), hmu.size() * 8, hipMemcpyHostToDevice));
    TCHK(hipMemcpy(dth, hth.data(), hth.size() * 8, hipMemcpyHostToDevice));
    TCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    TCHK(hipEventCreate(&e0));
    TCHK(hipEventCreate(&e1));
    Seq q;
    q.pl = plan;
    q.s = s;
    q.plain = 0;
    q.fp32 = 0;
    q.qmqm = 1;
    q.cells = 0;
    q.max_nq = q.total_nq = nq;
    q.max_nm = q.total_nm = n_mm;
    q.fa.frames = nullptr;
    q.fa.f0 = make_frame(plan->p.box, nq, n_mm, 0, 0, 0, plan->p.rcut);
    q.fa.n_frames = 1;
    st = seq_begin(q, dqp, dQ, dmu, dth, dm, dq, 2, 1);
    if (st != EWALD_OK) goto done;
    TCHK(launch_sfac_qm(plan->g, q.fa, nq, dQ, dmu, dth, plan->w.qeff, nullptr, 1, plan->w, s));
    auto time_it = [&](auto&& launch) -> double {
      hipError_t e = launch();  // warm-up
      if (e != hipSuccess) return -1.0;
      if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
      for (int r = 0; r < 3; r++)
        if (launch() != hipSuccess) return -1.0;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
      return 1e3 * ms / 3.0;
    };
    char item[160];
    struct FwdCand {
      int mode, ct, ft, xcd;
    };
    std::vector<FwdCand> fc;
    if (mfma_fwd_ok(plan->g))
      for (int ct : {1, 2, 4})
        if (saved.fp32r ? fp32r_ct_ok(plan->g, ct) : mfma_fwd_ct_ok(plan->g, ct))
          for (int ft : {512, 768, 1024, 1536, 2304})
            for (int xcd : {0, 1}) fc.push_back({1, ct, ft, xcd});
    if (!saved.fp32r)  // the FP32 variant has only the matrix-core forward
      for (int ft : {4096, 8192, 16384}) fc.push_back({0, 0, ft, 0});
    for (const FwdCand& c : fc) {
      plan->t = saved;
      plan->t.fwd_mode = c.mode;
      plan->t.fwd_xcd = c.xcd;
      if (c.mode == 1) plan->t.fwd_ct = c.ct;
      plan->t.fwd_target = c.ft;
      plan->t.a_chunk = 0;
      plan->t.a_chunk = choose_a_chunk(plan, {n_mm});
      const double us = time_it([&]() { return launch_sfac_mm(plan->g, plan->t, q.fa, n_mm, plan->cap_mm, plan->w, s); });
      if (us < 0) {
        st = fail(EWALD_ERR_HIP, "autotune: forward launch failed");
        goto done;
      }
      if (c.mode == 1)
        snprintf(item, sizeof(item), "%s\"fwd_mfma_ct%d_%d_x%d\": %.1f", report.empty() ? "" : ", ", c.ct, c.ft,
                 c.xcd, us);
      else
        snprintf(item, sizeof(item), "%s\"fwd_valu_%d\": %.1f", report.empty() ? "" : ", ", c.ft, us);
      report += item;
      fres.push_back({us, plan->t});
      if (us < best_f) {
        best_f = us;
        best.fwd_mode = c.mode;
        best.fwd_xcd = c.xcd;
        best.fwd_ct = c.mode == 1 ? c.ct : saved.fwd_ct;
        best.fwd_target = c.ft;
      }
    }
    for (int bw : {2, 3, 4, 5, 6}) {
      if (bw >= 3 && !mfma_bwd_ok(plan->g)) continue;
      if (bw == 6 && !mfma_bwd_eyl_ok(plan->g)) continue;
      if (saved.fp32r && bw != 6) continue;  // the FP32 variant has only the LDS-y adjoint
      for (int kc : {0, 1, 2, 3, 4, 5, 6, 8, 16})
        for (int bx : {0, 1}) {
          if (kc > plan->cap_kc || (bx == 1 && bw != 6)) continue;
          plan->t = saved;
          plan->t.bwd_ilp = bw;
          plan->t.bwd_xcd = bx;
          plan->t.kc = kc;
          plan->t.kc = choose_kc(plan, n_mm);
          const double us =
              time_it([&]() { return launch_force_mm(plan->g, plan->t, q.fa, n_mm, plan->cap_mm, plan->w, s); });
          if (us < 0) {
            st = fail(EWALD_ERR_HIP, "autotune: adjoint launch failed");
            goto done;
          }
          if (bw == 6)
            snprintf(item, sizeof(item), ", \"bwd%d_kc%d_x%d\": %.1f", bw, plan->t.kc, bx, us);
          else
            snprintf(item, sizeof(item), ", \"bwd%d_kc%d\": %.1f", bw, plan->t.kc, us);
          report += item;
          bres.push_back({us, plan->t});
          if (us < best_b) {
            best_b = us;
            best.bwd_ilp = bw;
            best.bwd_xcd = bx;
            best.kc = kc;
          }
        }
    }
    // In-context pick.  Inside the fused step the adjoint's blocks start while
    // the forward's drain, beside the QM-side kernels, and the standalone times
    // of close candidates do not rank their step times (a forward grid of one
    // full round can finish sooner but leave the adjoint a worse start): the
    // standalone finalists (within 3% of the best; the best block order of up
    // to three forward tilings and four adjoint chunkings) are timed as whole
    // forward+adjoint steps.
    {
      auto finalists = [](std::vector<std::pair<double, Tuning>> v, double b, size_t n, auto key) {
        std::stable_sort(v.begin(), v.end(),
                         [](const std::pair<double, Tuning>& x, const std::pair<double, Tuning>& y) {
                           return x.first < y.first;
                         });
        std::vector<Tuning> out;
        for (const auto& e : v) {
          if (e.first > 1.03 * b || out.size() >= n) break;
          bool seen = false;
          for (const Tuning& o : out) seen = seen || key(o) == key(e.second);
          if (!seen) out.push_back(e.second);
        }
        return out;
      };
      const std::vector<Tuning> ff = finalists(fres, best_f, 3, [](const Tuning& t) {
        return (long)t.fwd_mode * 1000000L + (long)t.fwd_ct * 100000L + t.fwd_target;
      });
      const std::vector<Tuning> bf =
          finalists(bres, best_b, 4, [](const Tuning& t) { return (long)t.bwd_ilp * 1000L + t.kc; });
      if (ff.size() * bf.size() > 1) {
        TCHK(hipMalloc(&d_out, sizeof(double) * (1 + 10 * (size_t)std::max(nq, 1))));
        TCHK(hipMalloc(&d_ctx, std::max<size_t>(ctx_bytes(plan->g, nq, n_mm), 256)));
        // the combinations are timed in interleaved rounds (drift of clocks and
        // of the other streams' timing affects all alike) and each keeps the
        // median of its rounds
        std::vector<Tuning> cands;
        for (const Tuning& a : ff)
          for (const Tuning& b : bf) {
            Tuning c = best;
            c.fwd_mode = a.fwd_mode;
            c.fwd_ct = a.fwd_ct;
            c.fwd_target = a.fwd_target;
            c.fwd_xcd = a.fwd_xcd;
            c.a_chunk = 0;
            c.bwd_ilp = b.bwd_ilp;
            c.bwd_xcd = b.bwd_xcd;
            c.kc = b.kc;
            cands.push_back(c);
          }
        constexpr int kRounds = 5;
        std::vector<std::vector<double>> times(cands.size());
        for (int rd = 0; rd < kRounds; rd++)
          for (size_t ci = 0; ci < cands.size(); ci++) {
            plan->t = cands[ci];
            const double us = time_it([&]() {
              const ewald_status_t r =
                  ewald_forward(plan, nq, dqp, dQ, dmu, dth, n_mm, dm, dq, d_out, d_out + 1, d_out + 1 + nq,
                                d_out + 1 + 4 * (size_t)nq, d_ctx, (void*)s);
              return r == EWALD_OK ? hipSuccess : hipErrorLaunchFailure;
            });
            plan->t = cands[ci];
            if (us < 0) {
              st = fail(EWALD_ERR_HIP, "autotune: step failed: %s", g_last_error.c_str());
              goto done;
            }
            times[ci].push_back(us);
          }
        double best_s = 1e30;
        Tuning pick = best;
        for (size_t ci = 0; ci < cands.size(); ci++) {
          std::vector<double> v = times[ci];
          std::sort(v.begin(), v.end());
          const double med = v[v.size() / 2];
          const Tuning& c = cands[ci];
          snprintf(item, sizeof(item), ", \"step_ct%d_%d_x%d_bwd%d_kc%d_x%d\": %.1f", c.fwd_ct, c.fwd_target,
                   c.fwd_xcd, c.bwd_ilp, c.kc, c.bwd_xcd, med);
          report += item;
          if (med < best_s) {
            best_s = med;
            pick = c;
          }
        }
        best = pick;
      }
    }
  }
done:
#undef TCHK
  plan->t = st == EWALD_OK ? best : saved;
  plan->t.a_chunk = 0;
  if (s) (void)hipStreamSynchronize(s);
  for (double* p : {dm, dq, dqp, dQ, dmu, dth, d_out})
    if (p) (void)hipFree(p);
  if (d_ctx) (void)hipFree(d_ctx);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (st != EWALD_OK) return st;
  set_describe(plan);
  if (cache_path) {
    FILE* fp = fopen(cache_path, "a");
    if (fp) {
      fprintf(fp,
              "{\"key\": \"%s\", \"fwd\": %d, \"ct\": %d, \"xcd\": %d, \"fwd_target\": %d, \"bwd\": %d, "
              "\"bxcd\": %d, \"kc\": %d, \"times_us\": {%s}}\n",
              key.c_str(), plan->t.fwd_mode, plan->t.fwd_ct, plan->t.fwd_xcd, plan->t.fwd_target, plan->t.bwd_ilp,
              plan->t.bwd_xcd, plan->t.kc, report.c_str());
      fclose(fp);
    }
  }
  return EWALD_OK;
}
