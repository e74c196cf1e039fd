/* mtp.h -- C ABI of the MI355X (gfx950) Moment Tensor Potential library.
 *
 * The library evaluates the per-neighborhood hot path of the Moment Tensor
 * Potential as used by MLIP-3 (Podryabinkin et al., arXiv 2304.13144):
 *
 *   neighborhoods n_i            (Sec. II.A, the tuple after eq. 1)
 *   radial functions f_mu        (eq. 4; Chebyshev polynomials, see below)
 *   moment tensors M_{mu,nu}     (eq. 3)
 *   basis functions B_alpha      (Sec. II.A, eqs. 5-6: contractions of moments)
 *   site / total energy          (eqs. 1-2)
 *   forces and stress            (the quantities fitted in eq. 7)
 *   rows b_i = dV(n_i)/dtheta    (Sec. II.D, eq. 10)
 *   grades gamma_i = max_p |(b_i A^-1)_p|          (Sec. II.D)
 *   MaxVol swaps into the active set A             (Sec. II.C)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value: an mtp_status; MTP_OK (0) on success.  No entry point aborts
 * or throws across the ABI; on error mtp_last_error() returns a message
 * (thread-local, valid until the next call on the same thread).  Inputs are
 * validated before any work is enqueued; outputs are untouched on a
 * validation error.
 *
 * Memory: every array argument is caller-owned DEVICE memory on the model's
 * device unless the comment says "host".  The library owns only the opaque
 * handles below and their internal workspaces (allocated on first use at a
 * given capacity, reused afterwards).
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  All work is enqueued on it; nothing synchronises unless the
 * comment says so.
 *
 * Units: Angstrom, eV, eV/Angstrom; stress in eV (not divided by volume).
 *
 * Parameter vector theta (FP64, length n_theta):
 *   [ xi_0 (n_types) | xi_1..xi_Nlin | c (N_rad, n_types, n_types, N_polyn) ]
 * xi_0 is one constant per species (the parameter counts of Sec. IV need it);
 * c[mu][z_i][z_j][beta] multiplies T_beta(x) (R_cut - r)^2 with T_beta the
 * Chebyshev polynomial of degree beta (beta = 0..N_polyn-1) and
 * x = (2 r - R_min - R_cut) / (R_cut - R_min).
 */
#ifndef MTP_H
#define MTP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MTP_OK = 0,
    MTP_E_INVAL = -1,       /* bad argument (NULL, size, enum, NaN/Inf input) */
    MTP_E_IO = -2,          /* model file cannot be read / written */
    MTP_E_PARSE = -3,       /* model file malformed */
    MTP_E_OVERLAP = -4,     /* two atoms closer than 1e-6 Angstrom */
    MTP_E_CAPACITY = -5,    /* a neighborhood has more than max_nbrs atoms */
    MTP_E_SINGULAR = -6,    /* active-set matrix not invertible */
    MTP_E_HIP = -7,         /* HIP runtime error */
    MTP_E_NOMEM = -8,       /* device allocation failed */
    MTP_E_UNSUPPORTED = -9  /* level / type count not compiled into the library */
} mtp_status;

typedef enum { MTP_FP64 = 0, MTP_MIXED = 1 } mtp_precision;
/* MTP_FP64: every step in double precision.
 * MTP_MIXED: pair gradients (the force and stress terms) in FP32 with FP64
 *   sums; energies, forces and stress only: radial functions, moments and
 *   contractions in FP32 too.  When grades or rows are asked for, the
 *   moments, contractions and rows run in FP64 (the grade amplifies row
 *   errors by the conditioning of A: FP32 rows miss gamma to 1e-5 on a
 *   level-16 active set) and the grade product is an int8 slice product
 *   on MFMA with exact int32 accumulation (m <= 320; FP64 MFMA beyond).
 *   A^-1 and MaxVol in FP64 in both forms. */

typedef enum {
    MTP_GRADE_FULL = 0,
    MTP_GRADE_LINEAR = 1,
    MTP_GRADE_FULL_CFG = 2,
    MTP_GRADE_LINEAR_CFG = 3
} mtp_grade_mode;
/* FULL: b_i over all of theta minus N_rad(N_rad+1)/2 gauge columns of the c
 *   block (the rows are exactly rank deficient by that many directions), so
 *   m = n_theta - N_rad(N_rad+1)/2.  LINEAR: b_i = (onehot(z_i), B_alpha),
 *   m = n_types + N_lin.
 * FULL_CFG / LINEAR_CFG: the query strategy on whole configurations (Sec.
 *   II.C): the row of a configuration is b(cfg) = dE/dtheta = sum_i b_i over
 *   its atoms (FULL or LINEAR columns), and the active set holds m such
 *   configuration rows.  Each of the four modes has an active set of its own
 *   (mtp_set_active_set, mtp_maxvol_update). */

typedef struct mtp_model mtp_model; /* theta, basis, A^-1 per mode (device) */
typedef struct mtp_nbrs mtp_nbrs;   /* neighbor lists of one system (device) */

typedef struct {
    int32_t level, n_types, n_polyn;
    int32_t n_lin;          /* number of basis functions B_alpha */
    int32_t n_rad;          /* number of radial functions f_mu */
    int32_t n_comp;         /* symmetric moment components per neighborhood */
    int32_t n_theta;        /* length of theta */
    int32_t m_full, m_linear;
    double r_min, r_cut;
    int32_t has_active_full, has_active_linear;
    int64_t contraction_flops;  /* flops of the contraction program per neighborhood */
} mtp_model_info;

/* A batch of configurations (all pointers device memory; pos and type may
 * be NULL when n_atoms is 0). */
typedef struct {
    int32_t n_cfg;
    int64_t n_atoms;
    const int64_t *cfg_off; /* [n_cfg+1] first atom of each configuration */
    const double *pos;      /* [n_atoms*3] Cartesian positions */
    const int32_t *type;    /* [n_atoms] species 0..n_types-1 */
    const double *cell;     /* [n_cfg*9] row k = cell vector k */
    const uint8_t *pbc;     /* [n_cfg*3] periodic flags, or NULL = all periodic */
} mtp_system;

/* --- model ------------------------------------------------------------ */

/* Reads a potential file and uploads it to `hip_device` (paper Sec. III.A:
 * the potential file carries the trained parameters together with the
 * active set, so that grades can be computed from the file alone).  The
 * format is the library's own text format, written by mtp_save, not the
 * paper's: level, species count, R_min, R_cut, N_polyn, theta (Sec. II.B
 * order: xi_0 per species, xi_alpha, c) and optionally the active sets.
 * Errors: MTP_E_INVAL (NULL argument), MTP_E_IO (unreadable file),
 * MTP_E_PARSE (malformed or inconsistent content), MTP_E_UNSUPPORTED
 * (level, species count or N_polyn not compiled in), MTP_E_HIP; *out is
 * untouched on error.  The caller frees the model with mtp_free. */
int mtp_load(const char *path, int hip_device, mtp_model **out);

/* Writes the model (host-side copy of theta and active sets) to `path`. */
int mtp_save(const mtp_model *m, const char *path);

/* A model with theta = 0 and no active set (level must be compiled in). */
int mtp_create(int32_t level, int32_t n_types, double r_min, double r_cut, int hip_device, mtp_model **out);

int mtp_free(mtp_model *m);
int mtp_info(const mtp_model *m, mtp_model_info *info /* host */);

/* Replaces theta (device FP64 [n_theta]); recomputes the FULL-mode gauge
 * columns from the new c (column-pivoted QR of [c_0;..;c_mu] per mu) and
 * invalidates the FULL active set (its rows depend on theta).  Synchronises
 * `stream` (the gauge choice is made on the host). */
int mtp_set_params(mtp_model *m, const double *theta, void *stream);

/* Copies theta (FP64 [n_theta]) to host memory. */
int mtp_get_params(const mtp_model *m, double *theta /* host */);

/* Columns of theta kept in FULL mode, ascending (host [m_full]). */
int mtp_kept_columns(const mtp_model *m, int32_t *cols /* host */);

/* Sets the active set of `mode` from its m x m row-major FP64 matrix
 * (device; rows = b rows of the active neighborhoods in that mode's column
 * space) and computes A^-1 in FP64 by Gauss-Jordan elimination with partial
 * pivoting.  Returns MTP_E_SINGULAR (after synchronising `stream`) if a
 * pivot falls below 1e-300 in magnitude. */
int mtp_set_active_set(mtp_model *m, mtp_grade_mode mode, const double *A, void *stream);

/* Copies A (rows of the active set) or A^-1 of `mode` to `out` (device m*m). */
int mtp_get_active_set(const mtp_model *m, mtp_grade_mode mode, double *A_out, double *Ainv_out, void *stream);

/* --- neighborhoods (Sec. II.A) ------------------------------------------ */

int mtp_nbrs_create(mtp_nbrs **out);
int mtp_nbrs_free(mtp_nbrs *nb);

/* Builds, for every atom i of every configuration, the list of (j, n) with
 * 0 < |x_j + n.H - x_i| < R_cut (n: integer image shifts, zero along
 * non-periodic axes).  Cell-list algorithm; lists are grouped by neighbor
 * species; the order inside a group is deterministic.  Capacity: max_nbrs
 * entries per atom.  Overflow and overlap are flagged on the device and
 * reported by mtp_nbrs_status. */
int mtp_build_neighbors(const mtp_model *m, const mtp_system *s, int32_t max_nbrs, mtp_nbrs *nb, void *stream);

/* Synchronises `stream`; returns MTP_OK, MTP_E_CAPACITY (with the largest
 * count in the message), MTP_E_OVERLAP, or MTP_E_INVAL (a position that is
 * not finite, a singular cell, a species out of range, an image shift past
 * +-127 cells) for the last build. */
int mtp_nbrs_status(const mtp_nbrs *nb, void *stream);

/* Copies the lists out: count [n_atoms] (int32), j [n_atoms*max_nbrs]
 * (int32), shift [n_atoms*max_nbrs*3] (int32); entries past count are
 * unspecified.  Any pointer may be NULL.  Returns max_nbrs in *stride. */
int mtp_nbrs_export(const mtp_nbrs *nb, int32_t *count, int32_t *j, int32_t *shift, int32_t *stride /* host */,
                    void *stream);

/* --- evaluation ----------------------------------------------------------- */

/* Energy per configuration (eqs. 1-2), forces F = -dE/dx, stress
 * S_ab = -dE/d eps_ab under x -> (I + eps) x (eV), site energies V_i.
 * energy [n_cfg], forces [n_atoms*3], stress [n_cfg*9] (row-major), site_e
 * [n_atoms] or NULL.  All FP64.  The neighbor lists must come from
 * mtp_build_neighbors on the same positions. */
int mtp_energy_forces_stress(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p,
                             double *energy, double *forces, double *stress, double *site_e, void *stream);

/* The same as mtp_energy_forces_stress, allocating nothing: for callers that
 * cannot call hipMalloc (code under HIP graph capture, tight serving or MD
 * loops, harnesses that forbid allocation).  Its scratch (moments, dE/dM,
 * pair gradients, per-atom virials and site energies, sum partials) is one
 * static device array of MTP_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends; a call whose evaluation needs more (about 2.4 KB per atom
 * at level 16 with max_nbrs 64 in FP64, so some 27,000 atoms) returns
 * MTP_E_CAPACITY before anything is enqueued.  The neighbor lists must
 * already be built.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller; nothing in the array needs to start at zero. */
#define MTP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mtp_energy_forces_stress_noalloc(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p,
                                     double *energy, double *forces, double *stress, double *site_e, void *stream);

/* Grades gamma_i = max_p |(b_i A^-1)_p| of every neighborhood (Sec. II.D)
 * and the argmax p (lowest on ties).  gamma [n_atoms] FP64, argmax
 * [n_atoms] int32 or NULL; b_rows (optional) receives the rows, [n_atoms*m]
 * row-major FP64 (both precisions).  Needs the mode's active set. */
int mtp_grade(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
              double *gamma, int32_t *argmax, void *b_rows, void *stream);

/* Grades of rows the caller holds (Sec. II.D): gamma_i = max_p |(b_i A^-1)_p|
 * and the argmax p (lowest on ties) for n rows b_i against the active set of
 * mode g (MTP_GRADE_FULL or MTP_GRADE_LINEAR), by the kernels and the tuned
 * kernel form of the fused evaluation.  rows (device, FP64, read only): the
 * evaluation's own column-major layout, entry (i, k) at rows[k * ld + i] with
 * ld >= n, for k < ldb, where ldb >= m rounded up to a multiple of 32
 * (MTP_FP64) or 64 (MTP_MIXED, whose int8 product steps k by 64) and the
 * columns m <= k < ldb hold zeros.  gamma [n] FP64 and argmax [n] int32 (or
 * NULL) on the device.  MTP_E_INVAL for a bad mode or precision, ld < n, a
 * short ldb or a mode without an active set. */
int mtp_grade_rows(const mtp_model *m, mtp_precision p, mtp_grade_mode g, const double *rows, int64_t n, int64_t ld,
                   int32_t ldb, double *gamma, int32_t *argmax, void *stream);

/* Configuration grades (Sec. II.C): gamma(cfg) = max_p |(b(cfg) A^-1)_p|
 * with b(cfg) = sum of the rows b_i of the configuration's atoms (FP64 rows
 * and sums in both precisions) and A the active
 * set of mode g (MTP_GRADE_FULL_CFG or MTP_GRADE_LINEAR_CFG; the product in
 * FP64 in both precisions).  gamma [n_cfg] FP64 and argmax [n_cfg] int32
 * (lowest p on ties) may be NULL when b_cfg is given; b_cfg [n_cfg*m] FP64
 * row-major or NULL.  gamma needs the mode's active set. */
int mtp_grade_cfg(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
                  double *gamma, int32_t *argmax, double *b_cfg, void *stream);

/* One fused pass: energy, forces, stress, site energies and grades (any
 * output pointer may be NULL; gamma needs the active set of `g`). */
int mtp_evaluate(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
                 double *energy, double *forces, double *stress, double *site_e, double *gamma, int32_t *argmax,
                 void *stream);

/* mtp_evaluate followed by the preselection of mtp_select (Sec. II.E) on the
 * grades just computed: idx [capacity] receives the i with gamma_i >
 * threshold in ascending order and *count (device int32) their number, at
 * most `capacity`.  The grade kernel counts the selected rows of each block
 * of rows as it writes gamma, so only the placement remains (one launch
 * instead of mtp_select's two), and that launch also gathers the forces and
 * finishes the per-configuration sums.  Results equal mtp_evaluate's bit for
 * bit.  gamma may be NULL (grades kept internally); needs the active set of
 * `g`.  idx and count must not be NULL. */
int mtp_evaluate_select(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p,
                        mtp_grade_mode g, double *energy, double *forces, double *stress, double *site_e,
                        double *gamma, int32_t *argmax, double threshold, int32_t *idx, int32_t capacity,
                        int32_t *count, void *stream);

/* FP64 rows b_i of the listed atoms only ([n_idx*m] row-major), e.g. the
 * candidates preselected by mtp_select for MaxVol. */
int mtp_b_rows(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_grade_mode g, const int32_t *idx,
               int32_t n_idx, double *rows, void *stream);

/* Preselection of extrapolative neighborhoods (Sec. II.E): writes the
 * indices i with gamma_i > threshold, ascending, to idx [capacity] and
 * their number to *count (device int32); at most `capacity` are written. */
int mtp_select(const double *gamma, int64_t n, double threshold, int32_t *idx, int32_t capacity, int32_t *count,
               void *stream);

/* MaxVol (Sec. II.C) in FP64: C = cand A^-1; while max |C_ij| > threshold
 * (> 1) and fewer than max_swaps swaps: row j of A <- candidate i, A^-1 and
 * C by rank-1 (Sherman-Morrison) updates, and the replaced row takes the
 * candidate's place in `cand` (so cand is modified in place).  Ties: lowest
 * i, then lowest j.  swap_cand / swap_col [max_swaps] device int32 receive
 * the log; *n_swaps (host) the number of swaps (synchronises `stream`). */
int mtp_maxvol_update(mtp_model *m, mtp_grade_mode g, double *cand, int64_t n_cand, double threshold,
                      int32_t max_swaps, int32_t *swap_cand, int32_t *swap_col, int32_t *n_swaps, void *stream);

/* --- extrapolation-controlled runs (Sec. II.F, Sec. III.A) ------------------ */

/* The spherical fragment around the atom of largest grade, for learning on
 * neighborhoods: that atom (the lowest index among equal maxima) and every
 * atom or periodic image strictly closer than `cutoff` (e.g. 8 A), as a
 * non-periodic cluster.  s: one configuration; grades: device [n_atoms]
 * (e.g. from mtp_grade).  Outputs (device, any may be NULL), ordered by
 * (source atom, image shift), at most `capacity` entries: pos_out [k*3]
 * (A, x_j + n.H in the frame of the cell), type_out [k], src_out [k] (source
 * atom), shift_out [k*3] (n).  *count (host) = entries written (the total
 * when it fits, else capacity); *center (host, may be NULL) = the central
 * atom.  Synchronises `stream`. */
int mtp_cut_neighborhood(const mtp_system *s, const double *grades, double cutoff, int32_t capacity, double *pos_out,
                         int32_t *type_out, int32_t *src_out, int32_t *shift_out, int32_t *count /* host */,
                         int32_t *center /* host */, void *stream);

/* Velocity-Verlet molecular dynamics (NVE; A, fs, amu, eV) with
 * extrapolation control: every configuration, the initial one included, is
 * graded before its forces are used, gamma(cfg) = max_i gamma_i in the
 * neighborhood mode g (FULL or LINEAR, needs its active set).  gamma(cfg) <=
 * gamma_save: go on; gamma_save < gamma(cfg) <= gamma_break: record the
 * step in saved[] and go on (no step when gamma_save >= gamma_break);
 * gamma(cfg) > gamma_break: stop (positions are
 * those of the graded step, velocities half-kicked).  One configuration;
 * pos must be s->pos (device [n_atoms*3], updated in place), vel device
 * [n_atoms*3] A/fs (updated); masses host [n_types] amu.  Neighbor lists
 * are rebuilt every step into nb with max_nbrs.  gamma_hist (host
 * [n_steps+1] or NULL) receives gamma(cfg) of steps 0..; saved (host
 * [n_steps+1] or NULL) the recorded steps, *n_saved their number;
 * *steps_done the completed steps (n_steps unless stopped).  Synchronises
 * `stream` every step (the grade decides whether to go on). */
int mtp_md_run(const mtp_model *m, const mtp_system *s, mtp_nbrs *nb, int32_t max_nbrs, double *pos, double *vel,
               const double *masses /* host */, double dt, int32_t n_steps, mtp_precision p, mtp_grade_mode g,
               double gamma_save, double gamma_break, double *gamma_hist /* host */, int32_t *saved /* host */,
               int32_t *n_saved /* host */, int32_t *steps_done /* host */, void *stream);

/* Structure relaxation with extrapolation control (Sec. III.A, the relax
 * command): FIRE (Bitzek et al., Phys. Rev. Lett. 97, 170201 (2006); the
 * paper names no minimizer).  Velocities start at zero; each step: stop if
 * max_i |F_i| < fmax (eV/A); P = F.v over all 3N components; if P > 0,
 * v <- (1 - alpha) v + alpha |v| F / |F| and, after more than 5 such steps
 * in a row, dt <- min(1.1 dt, dt_max), alpha <- 0.99 alpha; else v <- 0,
 * dt <- dt / 2, alpha <- 0.1 (alpha starts at 0.1, dt at dt0, fs); then
 * v <- v + dt F / m, x <- x + dt v.  Every configuration, the initial one
 * included, is graded before its forces are used, with the thresholds of
 * mtp_md_run (record between gamma_save and gamma_break, stop above).  One
 * configuration; pos must be s->pos (updated in place); masses host
 * [n_types] amu.  gamma_hist / saved / n_saved / steps_done as for
 * mtp_md_run; *converged (host) = 1 when the force tolerance was met. */
int mtp_relax_fire(const mtp_model *m, const mtp_system *s, mtp_nbrs *nb, int32_t max_nbrs, double *pos,
                   const double *masses /* host */, double dt0, double dt_max, double fmax, int32_t max_steps,
                   mtp_precision p, mtp_grade_mode g, double gamma_save, double gamma_break,
                   double *gamma_hist /* host */, int32_t *saved /* host */, int32_t *n_saved /* host */,
                   int32_t *steps_done /* host */, int32_t *converged /* host */, void *stream);

/* Fitting (Sec. II.B): minimizes the objective of eq. 7,
 *   L = sum_k [w_e (E_k - E_k^t)^2 + w_f sum_i |F_ik - F_ik^t|^2 + w_s sum_ab (S_abk - S_abk^t)^2],
 * over theta by BFGS on the inverse Hessian (FP64, host side; the energies,
 * forces, stresses and dL/dtheta on the device, as mtp_energy_forces_stress
 * and mtp_efs_backward).  Starting from the model's theta: d = -H g; the
 * step t is halved from t_0 until L(theta + t d) <= L + 1e-4 t g.d (at most
 * 40 halvings, else stop); t_0 = min(1, 0.1 / max|D g|) on the first
 * iteration, 1 after; s = t d, y = g_new - g; when y.s > 0, H (diag(D^2)
 * at first, D = scale (host [n_theta], the typical size of each parameter)
 * or 1 when scale is NULL, rescaled by y.s / y.H.y before the first update)
 * becomes (I - rho s y^T) H (I - rho y s^T) + rho s s^T, rho = 1 / y.s.
 * Stops when max |g| <= gtol or after max_iter iterations.  Targets: device E_t
 * [n_cfg], F_t [n_atoms*3], S_t [n_cfg*9] (NULL allowed where the weight
 * is 0).  The neighbor lists must be built for s.  On return the model holds
 * the last accepted theta (the FULL active sets are invalidated, as by
 * mtp_set_params); loss_hist (host [max_iter+1] or NULL) receives L at
 * every accepted iterate, *iters the number of iterations.  Synchronises
 * `stream` at every evaluation. */
int mtp_fit_bfgs(mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, const double *E_t,
                 const double *F_t, const double *S_t, double w_e, double w_f, double w_s, int32_t max_iter,
                 double gtol, const double *scale /* host */, double *loss_hist /* host */,
                 int32_t *iters /* host */, void *stream);

/* Gradient of the fitting objective (eq. 7) with respect to theta, given
 * the upstream gradients dL/dE [n_cfg], dL/dF [n_atoms*3], dL/dS [n_cfg*9]
 * (any may be NULL = 0): g_theta [n_theta] FP64.  Moments are recomputed;
 * no per-pair tensors are stored. */
int mtp_efs_backward(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, const double *gE,
                     const double *gF, const double *gS, double *g_theta, void *stream);

/* Kernel timing: while enabled, every library kernel group ("neighbors",
 * "efs", "force_gather", "cfg_sums", "grade", "select", "maxvol") is
 * bracketed by HIP events on its stream.  mtp_profile_read synchronises the
 * recorded events of `kernel`, returns their summed duration (ms) and count
 * and forgets them.  Host-side bookkeeping only; results are unaffected. */
int mtp_profile_enable(int on);
int mtp_profile_read(const char *kernel, double *total_ms /* host */, int64_t *launches /* host */);

/* Autotuner: times the evaluation of this system under nine schedules --
 * 2, 4 or 8 lanes per neighborhood for the moments / contraction (4 and 8:
 * one fused launch of four or eight wavefronts per 64 neighborhoods; 2: two
 * launches) and, independently, for the pair gradients -- (HIP events:
 * after a warm-up, five interleaved rounds of three evaluations per
 * schedule, each schedule's minimum), keeps the fastest for this model,
 * precision and size class (floor(log2 n_atoms)) and returns it in *lanes
 * (host) as 16 x (moments / contraction lanes) + (pair-gradient lanes).
 * Then, when the grade mode has an active set, it times the kernel forms of
 * the grade product (each form's launch alone, ten at a time, on the rows
 * the evaluations left, in five interleaved rounds) -- 1: FP64 MFMA with
 * each wavefront's rows in registers (m <= 288); 2: FP64 MFMA with the rows
 * staged through LDS (any m); 3: the int8 slice product (MTP_MIXED, m <=
 * 320); 4: as 1 in blocks of 32 rows, two blocks per CU (m <= 288); 5: FP64
 * MFMA with k outermost, the rows streamed in chunks of eight k steps beside
 * the products (m <= 288); 6: as 5 in chunks of two k steps, two blocks per
 * CU (m <= 288) -- keeps the fastest for this model, precision, grade mode
 * and size class and returns it in *grade (host, nullable; 0 when no grade was
 * timed).  Every form meets the precision's error bound; they differ in
 * speed only.  Synchronises `stream`. */
int mtp_tune(mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
             int32_t *lanes /* host */, int32_t *grade /* host, nullable */, void *stream);

/* Sustained MFMA rate of this GPU (measurement helper): a full grid of
 * eight wavefronts per CU runs four independent accumulation chains each of
 * one MFMA form on register operands (kind 0: v_mfma_f64_16x16x4, FP64;
 * kind 1: v_mfma_i32_16x16x64_i8) for `iters` iterations (rounded up to a
 * multiple of 16); *tflops (host)
 * receives the rate of the second of two launches in TFLOP/s (TOP/s for
 * int8).  The ceiling a kernel built on that form can reach, beside the
 * nominal peak.  Synchronises `stream`; MTP_E_INVAL for a bad kind or
 * iters outside 1 .. 2^24. */
int mtp_mfma_rate(int kind, int32_t iters, double *tflops /* host */, void *stream);

/* Description of the basis of a level, one function per line (host). */
int mtp_basis_describe(int32_t level, char *buf, size_t len, int32_t *n_lin);

/* Levels compiled into the library (host [cap]); returns how many. */
int mtp_compiled_levels(int32_t *levels, int32_t cap);

const char *mtp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MTP_H */
