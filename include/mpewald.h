/*
 * mpewald: periodic (Ewald) electrostatic coupling between atom-centred QM
 * point multipoles and MM point charges, on AMD Instinct MI355X (gfx950).
 *
 * Quantity (paper: Methods, "Multipole Approximation to Electrostatics",
 * the periodic QM/MM multipole energy; Supporting Information, "Multipolar
 * Ewald"):
 *
 *   E = E_QMMM + E_QQ
 *   E_QMMM = sum_j [ Q_j phi_j + mu_j . grad phi_j + theta_j : (1/2) grad grad phi_j ]
 *   phi(R) = sum_i q_i psi(R - R_i),  psi = Ewald kernel (real + reciprocal + background)
 *   E_QQ   = QM-QM image interactions truncated at total multipole order 2
 *            (charge-charge, charge-dipole, charge-quadrupole, dipole-dipole),
 *            including self terms; MM-MM interactions are excluded.
 *
 * Units: Coulomb constant 1.  Lengths and charges in any consistent units
 * (the tests use Angstrom and e, giving e^2/Angstrom).
 *
 * Conventions shared by every entry point:
 *   - All arrays are row-major, FP64, on the device of the plan, unless noted.
 *   - Positions: (N,3) [x,y,z per atom]; any real values (wrapped internally).
 *   - Dipoles mu: (Nq,3).  Quadrupoles theta: (Nq,6) raw Cartesian second
 *     moments (not traceless) stored as xx, xy, xz, yy, yz, zz; the 1/2 of
 *     the Taylor series is part of the order-2 interaction tensor.
 *   - phi: (Nq,) potential of the MM charges at each QM site;
 *     efield: (Nq,3) = -grad phi; efgrad: (Nq,6) = -grad grad phi (xx..zz).
 *   - Gradients are dE/dx (forces are minus these).  g_theta is the
 *     derivative with respect to the six stored numbers, so each stored
 *     off-diagonal number receives twice the full-matrix derivative.
 *   - Box: orthorhombic edges.  Real space sums every lattice image with
 *     |r| < rcut: only the minimum image when rcut <= min(box)/2, otherwise
 *     up to 3 images per direction (rcut below about 3.5 min(box); the
 *     paper's regime of a cutoff near the box length).  Reciprocal vectors are
 *     k = 2 pi (nx/Lx, ny/Ly, nz/Lz) for every |n_a| <= kmax[a], n != 0.
 *   - Boundary: tin-foil (no surface dipole term); uniform neutralising
 *     background for charged subsystems.
 *   - Streams: every call only enqueues work on `stream` (a hipStream_t,
 *     0 = default stream) and returns; no host synchronisation except in
 *     ewald_setup, ewald_autotune and the first ewald_batch call of a shape.
 *   - Errors: a negative status; arguments are validated on the host before
 *     anything is enqueued and outputs are left untouched on error.  The
 *     message of the last error of the calling thread is ewald_last_error().
 *   - Ownership: the caller owns every input, output and ctx buffer; the
 *     plan owns only its workspace, graphs and tuning state.  A plan must
 *     not be used by two host threads at once.
 */
#ifndef MPEWALD_H
#define MPEWALD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EWALD_OK = 0,
  EWALD_ERR_ARG = -1,      /* null pointer, bad size or bad parameter */
  EWALD_ERR_CUTOFF = -2,   /* rcut needs more than 3 lattice images per direction */
  EWALD_ERR_CAPACITY = -3, /* more atoms/frames than the plan was set up for, or a frame of more MM
                               charges than the matrix-core kernels address: 2^31 / (16 (kmax[0] + 2 kmax[1]
                               + 2)), 1.8 million at kmax 24 */
  EWALD_ERR_HIP = -4,      /* a HIP runtime call failed */
  EWALD_ERR_OOM = -5       /* workspace allocation failed */
} ewald_status_t;

/* precision (bit set; 0 = everything in FP64) */
enum {
  EWALD_FP64 = 0,          /* everything in FP64 */
  EWALD_FP32_REAL = 1,     /* real-space distances, erfc, exp and tensors in FP32,
                              accumulated in FP64 */
  EWALD_FP32_RECIP = 2     /* the two reciprocal-space hot loops (MM structure factor
                              and MM gradients) on FP32 matrix cores: phase tables and
                              folded weights rounded to FP32, FP32 accumulation inside
                              a block, FP64 sums across blocks and everything after;
                              needs kmax[2] <= 32 and kmax[1] <= 61.  The error against
                              FP64 is of the order of 1e-6 relative (mixed precision) */
};

/* flags */
enum {
  EWALD_QMQM = 1,          /* include the QM-QM image terms (on in the tests) */
  EWALD_PLAIN = 2,         /* forward uses the unoptimised reference GPU path:
                              one thread per k, direct sincos per (k, atom) */
  EWALD_CELL_LIST = 4,     /* real space visits only neighbouring cells */
  EWALD_PROFILE = 8,       /* time every kernel launch with events on its stream
                              (single-frame calls only; read with ewald_profile_report) */
  EWALD_PROFILE_HOT = 16,  /* as EWALD_PROFILE, but only the two reciprocal-space
                              hot loops (sfac_mm, force_mm): two events per launch */
  EWALD_NO_BACKGROUND = 32, /* leave out the uniform neutralising background of charged
                              subsystems, -(pi/(2 a^2 V)) Qtot^2 and -(pi/(a^2 V)) Qtot qtot,
                              which is included by default (the paper is silent on it;
                              neutral systems are unaffected) */
  EWALD_DETERMINISTIC = 64  /* bitwise reproducible results: every cross-block sum is
                              taken in a fixed order (per-block partial sums and a
                              fixed-order reduction) instead of with floating-point
                              atomics, and real space runs over all pairs (the cell
                              fill orders atoms with atomics).  Repeated calls with
                              the same plan, tiles and inputs return identical bytes;
                              the default mode differs from it by rounding only */
};

typedef struct {
  double box[3];   /* orthorhombic edges */
  double alpha;    /* Ewald splitting parameter (1/length), > 0 */
  double rcut;     /* real-space cutoff: pairs and lattice images with |r| < rcut */
  int kmax[3];     /* reciprocal cube |n_a| <= kmax[a], each >= 1 */
  int precision;   /* EWALD_FP64, or EWALD_FP32_REAL and/or EWALD_FP32_RECIP */
  int flags;       /* EWALD_QMQM | EWALD_PLAIN | EWALD_CELL_LIST | EWALD_PROFILE | EWALD_PROFILE_HOT |
                      EWALD_NO_BACKGROUND | EWALD_DETERMINISTIC */
  int max_qm;      /* capacity: QM sites per call (sum over frames in a batch) */
  int max_mm;      /* capacity: MM charges per call (sum over frames in a batch) */
  int max_frames;  /* capacity: frames per ewald_batch call (>= 1) */
} ewald_params_t;

typedef struct ewald_plan ewald_plan;

/* One frame of a batch: its box and where its atoms sit in the packed arrays. */
typedef struct {
  double box[3];
  int n_qm, n_mm;
  int qm_offset, mm_offset; /* first row of this frame in the packed QM / MM arrays */
} ewald_frame_t;

/* Create a plan on the current HIP device and allocate its workspace for
 * the given capacities.  The plan keeps a copy of *params: the Ewald
 * splitting parameter, real-space cutoff and k-space range of the multipolar
 * Ewald sums (paper: SI, Multipolar Ewald; Computational Details, Common
 * Setup, for the choice of the cutoff). */
ewald_status_t ewald_setup(const ewald_params_t* params, ewald_plan** plan);

/* Release the workspace of a plan made by ewald_setup; null is accepted. */
ewald_status_t ewald_destroy(ewald_plan* plan);

/* Change the box of a plan (validated like ewald_setup); affects later calls
 * (paper: Implementation, where the MD driver sends the box with every step). */
ewald_status_t ewald_set_box(ewald_plan* plan, const double box[3]);

/* Bytes of the caller-allocated context that ewald_forward fills and
 * ewald_backward reads (saved reciprocal structure factor of the MM charges
 * and the MM potential data at the QM sites: the MM field that the SCF
 * iterations and the gradient reuse, paper: Electronic Mean-Field Theory). */
size_t ewald_ctx_bytes(const ewald_plan* plan, int n_qm, int n_mm);

/* Forward pass (paper: periodic multipole energy; SI multipolar Ewald).
 * Inputs qm_xyz (Nq,3), Q (Nq), mu (Nq,3), theta (Nq,6), mm_xyz (Nm,3), mm_q (Nm).
 * Outputs energy (1), phi (Nq), efield (Nq,3), efgrad (Nq,6); any output
 * pointer except energy may be null.  ctx: null, or ewald_ctx_bytes() bytes
 * of device memory for a later ewald_backward.  n_qm or n_mm may be 0. */
ewald_status_t ewald_forward(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* Q, const double* mu,
                             const double* theta, int n_mm, const double* mm_xyz, const double* mm_q,
                             double* energy, double* phi, double* efield, double* efgrad, void* ctx, void* stream);

/* Adjoint of ewald_forward (paper: Fock-coupling potential v = dE/d(moments)
 * and the tensor part of the nuclear gradient; MM atoms have no Pulay term).
 * Upstream gradients: gE (device scalar, null means 1), g_phi (Nq), g_efield
 * (Nq,3), g_efgrad (Nq,6) (each may be null = zero).  Inputs as in forward,
 * ctx as filled by the matching forward call.
 * Outputs (overwritten): g_qm_xyz (Nq,3), g_Q (Nq), g_mu (Nq,3), g_theta (Nq,6),
 * g_mm_xyz (Nm,3), g_mm_q (Nm, may be null).  Each output is the gradient of
 * L = gE*E + g_phi.phi + g_efield.efield + g_efgrad.efgrad.
 * With upstream gradients on E only, the gradients that the forward call
 * stored in ctx are scaled by gE (one short kernel); after an
 * ewald_moments_update call on the same ctx (new moments at the same
 * geometry) the full adjoint runs instead, for the moments passed here. */
ewald_status_t ewald_backward(ewald_plan* plan, const void* ctx, int n_qm, const double* qm_xyz, const double* Q,
                              const double* mu, const double* theta, int n_mm, const double* mm_xyz,
                              const double* mm_q, const double* gE, const double* g_phi, const double* g_efield,
                              const double* g_efgrad, double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta,
                              double* g_mm_xyz, double* g_mm_q, void* stream);

/* Ewald parameters for a target accuracy (paper: Computational Details, the
 * Ewald parameters are estimated for a given accuracy with a real-space cutoff
 * of about the box length).  Given box and rcut, returns the smallest alpha
 * whose real-space truncation tail at rcut is below tol, and per axis the
 * smallest kmax whose reciprocal tail at k = 2 pi kmax / L is below tol.  The
 * tails are those of the order-2 screened tensors relative to the unscreened
 * term: erfc(a r) + (2/sqrt(pi)) a r e^{-a^2 r^2} (1 + 2/3 (a r)^2) and
 * e^{-k^2/4a^2} (1 + k^2/4a^2).  tol in (0, 0.1).  Host only; no plan needed. */
ewald_status_t ewald_suggest_params(const double box[3], double rcut, double tol, double* alpha, int kmax[3]);

/* Moments-only update for self-consistent-field iterations (paper: Electronic
 * Mean-Field Theory: the SCF iterates the QM density, hence the moments, at
 * fixed geometry, and needs E and the Fock-coupling potential v = dE/d(moments)
 * each iteration).  ctx must have been filled by ewald_forward with the same
 * plan, the same QM and MM positions and the same MM charges; only Q, mu and
 * theta may differ.  The MM field at the QM sites stored in ctx is reused and
 * only the QM-QM image terms (all k and real space, order-2 truncated) are
 * recomputed.  Outputs: energy (1, device), and, each may be null, g_Q (Nq),
 * g_mu (Nq,3), g_theta (Nq,6) = dE/d(moments) as in ewald_backward with gE = 1.
 * n_mm is the MM count of the forward call (it fixes the ctx layout).
 * Forces are not produced (positions are fixed); a later ewald_backward on
 * this ctx computes them, and every other gradient, for the moments it is
 * given (the plan remembers that the stored gradients no longer apply). */
ewald_status_t ewald_moments_update(ewald_plan* plan, const void* ctx, int n_qm, const double* qm_xyz,
                                    const double* Q, const double* mu, const double* theta, int n_mm,
                                    double* energy, double* g_Q, double* g_mu, double* g_theta, void* stream);

/* Region-I / region-II split (paper: Methods, the periodic QM/MM multipole
 * energy as whole-lattice Ewald sums minus direct sums over region I, and the
 * correction for Gaussian-smeared MM charges; SI: bare tensors T..T_abc and
 * screened ones with f1, f3, f5, f7 at kappa_i).  Region I is the sphere of
 * radius r_region around the arithmetic mean C of the QM positions; the QM
 * atoms of the cell belong to it, their periodic images do not.  The added
 * terms turn the outputs of ewald_forward into the region-II quantities that
 * the SCF uses (energy E^II and the potential v^II = dE^II/d(moments)):
 *   - the bare unit-cell QM-QM pairs: -1/2 sum_{a != b} P_T(a, b), the pair
 *     form of the QM-QM image terms with bare tensors, r = R_a - R_b with the
 *     QM positions as passed (not wrapped);
 *   - every lattice translate R_i + n L of every MM charge with
 *     |R_i + n L - C| < r_region: -q_i [Q T + mu.T_a + theta:T_ab] at each QM
 *     site (the sphere may exceed the cell; several translates of one atom
 *     may take part);
 *   - for MM charges with mm_kappa[i] > 0 (Gaussian charges of exponent
 *     kappa_i; mm_kappa null or <= 0: point charges): every translate outside
 *     the sphere within r_gauss of a QM site: -q_i [Q That + mu.That_a +
 *     theta:That_ab] with the tensors of erfc(kappa_i r)/r.
 * Box: the plan's.  r_region, r_gauss: >= 0 and at most 4 box lengths
 * (EWALD_ERR_CUTOFF otherwise).  Arrays as in ewald_forward, plus mm_kappa
 * (Nm) on the device.  n_qm and n_mm may not exceed the plan's max_qm and
 * max_mm.
 *
 * ewald_region_forward ADDS the region terms to energy (required), phi,
 * efield and efgrad (each may be null), e.g. to the outputs of an
 * ewald_forward call on the same stream.  ewald_region_backward ADDS the
 * gradient of L = gE E_r + g_phi.phi_r + g_efield.efield_r + g_efgrad.efgrad_r
 * of the region terms (gE device scalar, null = 1; the g_* may be null = 0) to
 * g_qm_xyz, g_Q, g_mu, g_theta, g_mm_xyz (required when the count is > 0) and
 * g_mm_q (may be null), e.g. after an ewald_backward call with the same
 * upstream gradients.  No gradient with respect to mm_kappa.  Calls on one
 * plan share a workspace: do not overlap them on different streams. */
ewald_status_t ewald_region_forward(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* Q,
                                    const double* mu, const double* theta, int n_mm, const double* mm_xyz,
                                    const double* mm_q, const double* mm_kappa, double r_region, double r_gauss,
                                    double* energy, double* phi, double* efield, double* efgrad, void* stream);
ewald_status_t ewald_region_backward(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* Q,
                                     const double* mu, const double* theta, int n_mm, const double* mm_xyz,
                                     const double* mm_q, const double* mm_kappa, double r_region, double r_gauss,
                                     const double* gE, const double* g_phi, const double* g_efield,
                                     const double* g_efgrad, double* g_qm_xyz, double* g_Q, double* g_mu,
                                     double* g_theta, double* g_mm_xyz, double* g_mm_q, void* stream);

/* Charge-octupole error estimate and R_cut search (paper: Error Control:
 * the leading error of the quadrupole-truncated multipole expansion is the
 * interaction of the region-II charges with the QM octupoles; R_cut is raised
 * in fixed steps from a lower bound until two consecutive values give an
 * estimate below the target accuracy; SI: T_abc = 1/3 d/dR_c T_ab).
 * For the candidates R_k = r_first + k r_step, k < n_r (1 <= n_r <= 256):
 *   err[k] = sum over MM translates R_i + n L with R_k <= |R_i + n L - C| < r_outer
 *            of q_i sum_j sum_abc Omega_j,abc T_abc(R_j - R_i - n L),
 * C the mean QM position.  omega (Nq,10): raw (not traceless) third moments
 * of the QM sites, xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz.  The sum
 * over region II converges absolutely and is truncated at r_outer (at most 4
 * box lengths, EWALD_ERR_CUTOFF otherwise).  r_cut (device scalar, may be
 * null) receives the first R_k with |err[k]| < eps and |err[k+1]| < eps, or -1
 * if no two consecutive candidates pass.  eps is in the energy unit of the
 * library (Coulomb constant 1: e^2/length).  n_mm may not exceed the plan's
 * max_mm.  err and r_cut are overwritten; device arrays. */
ewald_status_t ewald_octupole_error(ewald_plan* plan, int n_qm, const double* qm_xyz, const double* omega,
                                    int n_mm, const double* mm_xyz, const double* mm_q, int n_r, double r_first,
                                    double r_step, double r_outer, double eps, double* err, double* r_cut,
                                    void* stream);

/* Allocation-free variant of ewald_octupole_error, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): no plan; the box (3 orthorhombic edges,
 * host array) is passed directly and every other argument is as in
 * ewald_octupole_error.  The block partial sums of the estimate live in a
 * fixed array of the library in device memory (8 MiB, one copy per GPU, kept
 * until the process ends; its address is looked up on the first call on each
 * device), so the call allocates nothing.  Limit: n_r * ceil(n_mm / 256) <=
 * 1048576 (EWALD_ERR_CAPACITY beyond).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (different streams, or host threads)
 * race and must be ordered by the caller.  Each call writes every partial sum
 * it reads, so nothing carries over from the previous call. */
ewald_status_t ewald_octupole_error_noalloc(const double box[3], int n_qm, const double* qm_xyz, const double* omega,
                                            int n_mm, const double* mm_xyz, const double* mm_q, int n_r,
                                            double r_first, double r_step, double r_outer, double eps, double* err,
                                            double* r_cut, void* stream);

/* Batched evaluation of many independent frames with the plan's alpha, rcut
 * and kmax and per-frame boxes: per frame the computation of ewald_forward
 * and, with EWALD_FWD_BWD, of ewald_backward (paper: SI, Multipolar Ewald;
 * Results and Discussion, Timings, where the cost is the wall time per MD
 * step).  frames: host array of n_frames descriptors.
 * Packed inputs hold each frame's rows at its offsets.  mode: EWALD_FWD or
 * EWALD_FWD_BWD.  Outputs: energy (n_frames), phi/efield/efgrad per QM row;
 * with EWALD_FWD_BWD also dE/dx for every input (gE = 1): g_qm_xyz, g_Q,
 * g_mu, g_theta per QM row, g_mm_xyz and g_mm_q (may be null) per MM row.
 * The launch sequence of one frame shape is captured once in a HIP graph and
 * replayed while shapes, pointers and stream stay the same. */
enum { EWALD_FWD = 0, EWALD_FWD_BWD = 1 };
ewald_status_t ewald_batch(ewald_plan* plan, int n_frames, const ewald_frame_t* frames, const double* qm_xyz,
                           const double* Q, const double* mu, const double* theta, const double* mm_xyz,
                           const double* mm_q, int mode, double* energy, double* phi, double* efield, double* efgrad,
                           double* g_qm_xyz, double* g_Q, double* g_mu, double* g_theta, double* g_mm_xyz,
                           double* g_mm_q, void* stream);

/* Time the candidate tilings of the two reciprocal-space kernels for a
 * system of n_mm MM charges (synthetic, with the plan's QM capacity up to 64
 * sites) on the plan's device: each kernel alone, then the finalists within
 * 3% of the best as whole forward+adjoint steps in interleaved rounds; keep
 * the fastest step in the plan (and in cache_path as JSON lines if not null;
 * a later call with the same key reads it instead).  Allocates its own
 * scratch inputs and streams and synchronises.  n_mm outside 1..max_mm, or a
 * frame too large for the kernels' 32-bit offsets: EWALD_ERR_CAPACITY. */
ewald_status_t ewald_autotune(ewald_plan* plan, int n_mm, const char* cache_path);

/* Per-kernel launch counts and summed durations (ms) since the last report,
 * as a JSON object, for plans created with EWALD_PROFILE (for benchmark
 * reports).  Synchronises on the recorded events.  Returns EWALD_ERR_ARG if
 * len is too small. */
ewald_status_t ewald_profile_report(ewald_plan* plan, char* buf, size_t len);

/* Tile configuration in use (for reports): forward nz chunk, backward
 * columns per block, etc., as a short text. */
const char* ewald_plan_describe(const ewald_plan* plan);

/* Message of the calling thread's last error ("" if none); every entry point
 * that returns a status other than EWALD_OK sets it. */
const char* ewald_last_error(void);

/* Library version string. */
const char* ewald_version(void);

/* FP64 throughput probe (a diagnostic beside the published peaks, for
 * roofline reports): kind 0 issues back-to-back v_mfma_f64_16x16x4
 * instructions in four independent accumulator chains per wave, kind 1 FP64
 * VALU fused multiply-adds in eight independent chains per lane; blocks of
 * 256 threads, iters iterations each.  out: device buffer of at least
 * 4 * blocks doubles (one value per wave, written so no chain is optimised
 * away; caller-owned); *flops (host) receives the flops of the launch.
 * Asynchronous on stream; the caller times it.  Bad kind, blocks outside
 * 1..65536, iters outside 1..1e7 or a null pointer: EWALD_ERR_ARG. */
ewald_status_t ewald_fp64_probe(int kind, int blocks, int iters, double* out, double* flops, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MPEWALD_H */
