// Internal state and launch interfaces of libmtp (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mtp.h"
#include "basis.hpp"
#include "kernel_args.hpp"

namespace mtp {

// ---- errors ---------------------------------------------------------------
void set_error(const std::string &msg);
struct Error {
    int code;
    std::string msg;
};
#define MTP_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            throw ::mtp::Error{MTP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};      \
    } while (0)
#define MTP_CHECK(cond, code, msg)                                                                 \
    do {                                                                                           \
        if (!(cond)) throw ::mtp::Error{(code), (msg)};                                            \
    } while (0)

// ---- device buffers -------------------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    void ensure(size_t n);   // grows (no shrink); contents not preserved
    void release();
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

void launch_zero(void *p, size_t bytes, hipStream_t st);


struct ActiveSet {
    int m = 0;
    bool valid = false;
    DevBuf A;        // m*m FP64 rows
    DevBuf Ainv;     // m*m FP64
    // mixed-form product (see grade.hip): int8 digits of D^-1 A^-1
    // [GI_SL][CP8][KP8], their column exponents [CP8], the column scales D [KP8]
    DevBuf s8, fexp, dsc;
    int KP8 = 0, CP8 = 0;
    // FP64 product (m <= 320): A^-1 in the lane order of the grade kernel
    DevBuf lane64;
    int NK64 = 0;
};

// the kernels' copies of the ABI's enum values
static_assert(GRADE_FULL == MTP_GRADE_FULL && PREC_FP64 == MTP_FP64, "enum values");

}  // namespace mtp

struct mtp_model {
    int device = 0;
    int level = 0, n_types = 0;
    double r_min = 0, r_cut = 0;
    mtp::Basis basis;
    int n_theta = 0;
    std::vector<double> theta_host;
    std::vector<int> kept;          // FULL-mode kept columns
    std::vector<int> colmap_host;   // full column -> kept column or -1
    mtp::DevBuf theta64, theta32, colmap;
    mtp::ActiveSet act[4];          // indexed by mtp_grade_mode: neighborhood and configuration modes
    // schedules: 16 x (lanes of the moments / contraction) + (lanes of the pair gradients)
    int force_lanes = 0;            // set while the tuner times a schedule
    int tuned_lanes[2][48] = {};    // [precision][floor(log2 n_atoms)] -> schedule, 0 = untuned
    int force_grade = 0;            // set while the tuner times a grade schedule
    int tuned_grade[2][2][48] = {}; // [precision][grade mode][floor(log2 n_atoms)] -> GRADE_*, 0 = untuned
    // scratch of the evaluation path
    mutable mtp::DevBuf gbuf, virial, sitebuf, brow, gamma_ws, argmax_ws, work, sums, mbuf, dmbuf, tbuf, dtbuf, rows;
    mutable mtp::DevBuf selblk;     // per-block preselection counts written by the grade kernels
    mutable mtp::DevBuf gval, dgval;   // staged levels: graph values and dV/dg between the launches
    mutable mtp::DevBuf cfgrows, cfgpart;   // configuration-mode rows and their chunk partials
    mutable mtp::DevBuf md_f, md_g, md_invm, md_scal;   // MD driver: forces, grades, 1/mass, {gamma max, norms}
    mutable mtp::DevBuf md_v;                           // relaxation: FIRE velocities
    mutable mtp::DevBuf fit_y, fit_g, fit_part, fit_th;  // fitting: E/F/S, dL/d(E/F/S), loss partials, dL/dtheta
    // the configuration modes use the rows of their neighborhood mode (mode & 1)
    int m_of(int mode) const { return (mode & 1) == MTP_GRADE_FULL ? (int)kept.size() : n_types + basis.n_lin(); }
};

struct mtp_nbrs {
    int device = -1;
    int64_t n_atoms = 0;
    int32_t n_cfg = 0;
    int max_nbrs = 0, n_types = 0;
    double r_cut = 0;
    mtp::DevBuf r;        // [N*maxn*3] FP64 r_ij
    mtp::DevBuf j;        // [N*maxn] int32
    mtp::DevBuf shift;    // [N*maxn] int32 packed (3 x int8, x in the low byte; top byte: opposite bin offset)
    mtp::DevBuf pre;      // [N*n_types*64] uint16 list position where each bin offset's run starts
    mtp::DevBuf rev;      // [N*maxn] int32 flat index of (j, i, -n)
    mtp::DevBuf tcnt;     // [N*n_types] int32 neighbors per species
    mtp::DevBuf atom_cfg; // [N] int32
    mtp::DevBuf cfg_geo;  // per cfg geometry (see neighbors.hip)
    mtp::DevBuf bin_count, bin_start, bin_cursor, bin_atoms, atom_bin, atom_wrap;
    // atoms in bin order: position wrapped into the cell, packed -wrap, species
    mtp::DevBuf stage_x, stage_w, stage_t;
    mtp::DevBuf flags;    // [4] int32: overflow, max count, overlap, spare
    int64_t bins_cap = 0;
};

namespace mtp {

// ---- launchers (argument blocks in kernel_args.hpp) ------------------------
int launch_efs(int level, const EfsArgs &a);

int launch_backward(int level, const BwdArgs &b);
void launch_column_sums(const void *rows, int precision, int64_t n, int ncol, double *out, hipStream_t st,
                        DevBuf &work);
std::vector<int> compiled_levels();
long contraction_flops(int level);   // per neighborhood, from the generated program
int staged_graphs(int level);        // connected graphs of a level compiled as a staged program, else 0

void build_neighbors(const mtp_model *m, const mtp_system *s, int max_nbrs, mtp_nbrs *nb, hipStream_t st);

// Energy / stress per configuration (eq. 1) in two steps: partial sums over
// chunks of 32 atoms (written by the force gather when `part` is given, else
// by launch_cfg_partials), then one block per configuration.
void launch_force_gather(const mtp_nbrs *nb, const void *gbuf, int precision, double *forces, hipStream_t st,
                         const double *site_e = nullptr, const double *virial = nullptr, double *part = nullptr);
size_t cfg_partials_bytes(int64_t n_atoms);
void launch_cfg_partials(int64_t n, const double *site_e, const double *virial, double *part, hipStream_t st);
void launch_cfg_final(const mtp_system *s, const double *site_e, const double *virial, const double *part,
                      double *energy, double *stress, hipStream_t st);

// grade: C = b Ainv, gamma/argmax per row; b FP64 column-major (entry (i, k)
// at brow[k * ldn + i], ldb >= m columns, zero past m).  FP64 MFMA for the
// FP64 form, the exact int8 slice product for the mixed form (m <= 320;
// beyond, FP64).  thr / sel_blk (nullable): the grade also writes, per block
// of GRADE_ROWS rows, how many have gamma > thr (input of launch_select_write)
constexpr int GRADE_ROWS = 64;
// grade schedules (kernel forms): GRADE_AUTO picks by precision and m;
// GRADE_F64_REG: FP64 MFMA with the rows in registers (m <= 288);
// GRADE_F64_LDS: FP64 MFMA with the rows staged through LDS (any m);
// GRADE_I8: the int8 slice product (mixed form, m <= 320);
// GRADE_F64_PAIR: as GRADE_F64_REG in blocks of 32 rows, two blocks per CU;
// GRADE_F64_KOUTER: FP64 MFMA with k outermost, the rows streamed in chunks
// of eight k steps (m <= 288; one block per CU); GRADE_F64_KOUTER2: the same
// in chunks of two k steps (two blocks per CU)
enum {
    GRADE_AUTO = 0,
    GRADE_F64_REG = 1,
    GRADE_F64_LDS = 2,
    GRADE_I8 = 3,
    GRADE_F64_PAIR = 4,
    GRADE_F64_KOUTER = 5,
    GRADE_F64_KOUTER2 = 6
};
bool grade_sched_valid(const ActiveSet &as, int precision, int sched);
// rows per preselection count the grade writes under a schedule (divides GRADE_ROWS)
int grade_count_rows(const ActiveSet &as, int precision, int sched);
void launch_grade(const ActiveSet &as, int precision, const double *brow, int ldb, int64_t ldn, int64_t n,
                  double *gamma, int32_t *argmax, hipStream_t st, double thr = 0.0, int32_t *sel_blk = nullptr,
                  int sched = GRADE_AUTO);
void prepare_split(ActiveSet &as, hipStream_t st);
double mfma_rate(int kind, int iters, hipStream_t st);   // TFLOP/s (TOP/s) sustained; synchronises st
bool slice_product_fits(int m);
void launch_invert(ActiveSet &as, const double *A, hipStream_t st, DevBuf &work, int *singular_host);
void launch_select(const double *gamma, int64_t n, double thr, int32_t *idx, int32_t cap, int32_t *count,
                   hipStream_t st, DevBuf &work);
// the write half of the preselection, given per-GRADE_ROWS-block counts in
// blk [nb + 1] (overwritten with offsets when nb is large); with `sums` the
// same launch also finishes the configuration sums (launch_cfg_final)
struct CfgSums {
    const mtp_system *s;
    const double *site_e, *virial, *part;
    double *energy, *stress;
};
// the force gather as extra blocks of the same launch (forces from the pair
// gradients; independent of the grade)
struct GatherArgs {
    int64_t n = 0;
    int nt = 0, maxn = 0;
    const int32_t *tcnt = nullptr;
    const void *g = nullptr;
    int precision = 0;
    double *F = nullptr;
    int64_t blocks = 0;
};
GatherArgs gather_args(const mtp_nbrs *nb, const void *gbuf, int precision, double *forces);
void launch_select_write(const double *gamma, int64_t n, double thr, int32_t *blk, int32_t *idx, int32_t cap,
                         int32_t *count, hipStream_t st, const CfgSums *sums = nullptr,
                         const GatherArgs *gather = nullptr, int count_rows = GRADE_ROWS);
void run_maxvol(ActiveSet &as, double *cand, int64_t n_cand, double thr, int max_swaps, int32_t *swap_cand,
                int32_t *swap_col, int32_t *n_swaps, hipStream_t st, DevBuf &work);
// column-major rows (entry (i, k) at src[k * ldn + i]) -> row-major dst [n][m]
void launch_copy_rows(const double *src, int64_t ldn, int m, int64_t n, double *dst, hipStream_t st);
// extrapolation-controlled runs: largest value and its lowest index (one
// block; either output may be NULL); velocity-Verlet half steps (half 0:
// kick and drift, 1: kick); the spherical fragment around the largest
// grade: argmax, candidate keys over atoms x image shifts, ordered
// compaction, gather.  H: host cell (rows = lattice vectors), per: host pbc.
void launch_argmax(const double *g, int64_t n, double *best, int32_t *where, hipStream_t st);
void launch_md_step(int half, int64_t n, double *x, double *v, const double *F, const int32_t *type,
                    const double *inv_m, double h, double dt, hipStream_t st);
// FIRE: out [4] = {F.v, F.F, v.v, max_i |F_i|^2}; v <- a v + b F
void launch_fire_norms(int64_t n, const double *F, const double *v, double *out, hipStream_t st);
void launch_fire_mix(int64_t n, double *v, const double *F, double a, double b, hipStream_t st);
int64_t cut_fragment(const double *pos, const int32_t *type, int64_t n, const double *H, const int *per,
                     const double *g, double cutoff, int32_t cap, double *pos_out, int32_t *type_out,
                     int32_t *src_out, int32_t *shift_out, int32_t *count_dev, int32_t *center_dev, hipStream_t st,
                     DevBuf &keys, DevBuf &idx, DevBuf &work);
// fitting: g = 2 w (y - t) and per-256-entry partial sums of w (y - t)^2
// (returns the number of partials)
int64_t launch_fit_residual(int64_t n, const double *y, const double *t, double w, double *g, double *part,
                            hipStream_t st);
// configuration-mode rows: out (column-major, entry (c, k) at out[k * n_cfg + c])
// = per-configuration sums of the column-major FP64 rows (entry (i, k) at
// rows[k * n + i], ldb columns); part: cfg_row_partials_bytes(n, ldb)
size_t cfg_row_partials_bytes(int64_t n, int ldb);
void launch_cfg_rows(const double *rows, int ldb, int64_t n, const mtp_system *s, double *part, double *out,
                     hipStream_t st);
void launch_zero(void *p, size_t bytes, hipStream_t st);

// The fixed scratch region of the no-allocation entry point (a static device
// array, one copy per GPU): its device address on `device`, looked up once
// per device (that device must be current on the first call).
constexpr size_t NOALLOC_SCRATCH_BYTES = MTP_NOALLOC_SCRATCH_BYTES;
void *noalloc_scratch(int device);

}  // namespace mtp
