// Argument blocks of the evaluation and backward kernels, the constants they
// are compiled with and the launch profiler's scope guard: everything the
// per-level translation units need from the host side (kept apart from the
// library's host header so that host-only changes do not recompile them).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mtp {

constexpr int NPOLY = 8;     // Chebyshev polynomials per radial function
constexpr int MAX_TYPES = 4;
constexpr int GRADE_FULL = 0;   // = MTP_GRADE_FULL
constexpr int PREC_FP64 = 0;    // = MTP_FP64

struct EfsArgs {
    int64_t n_atoms;          // atoms processed (= list length if atom_list)
    const int32_t *atom_list; // optional: process these atoms
    int n_types, max_nbrs;
    const double *r;          // pair vectors
    const int32_t *tcnt;
    const int32_t *type;
    double r_min, r_cut;
    const double *th64;       // theta = [xi_0 | xi_alpha | c] in FP64
    const float *th32;        // and rounded to FP32
    int n_lin;
    // outputs (nullable)
    double *site_e;           // [n_atoms]
    void *gbuf;               // [N*maxn*3] T: pair gradient dV_i/dr_ij stored at the reverse pair's slot
    const int32_t *rev;       // [N*maxn] the reverse pair's slot (with gbuf)
    double *F;                // [N*3] with gbuf: sum_j dV_i/dr_ij per atom (the gather subtracts the rest)
    double *virial;           // [n_atoms*9]
    double *brow;             // rows b_i, FP64, column-major: entry (i, k) at brow[k * ldn + i]
    int64_t ldn;              // column stride of brow (>= n_atoms)
    int ldb;                  // columns written: m, then zeros up to ldb
    int grade_mode;           // rows layout: FULL (with colmap) or LINEAR
    const int32_t *colmap;    // full column -> kept column or -1
    int m;                    // row length written (kept columns)
    int precision;
    int lanes;                // lanes per neighborhood of the pair-gradient / row kernel (2, 4, 8)
    int lanes_mc;             // lanes per neighborhood of the moments / contraction (2, 4, 8; 4 = one launch)
    void *mbuf, *dmbuf;       // [NC][n_atoms] T: moments and dV/dM between the kernels
    void *gval, *dgval;       // staged levels only: [NGRAPH][n_atoms] T graph values and dV/dg
    // optional (atom_list NULL only): the pair-gradient blocks also write the
    // per-32-atom partial sums of part_e (V_i, nullable) and virial into part
    double *part;
    const double *part_e;
    hipStream_t stream;
};
struct BwdArgs {
    EfsArgs e;                // neighbors, parameters, mbuf (moments), dmbuf (dV/dM)
    const double *gE, *gF, *gS;
    const int32_t *atom_cfg;
    const int32_t *nbr_j;
    void *tbuf, *dtbuf;       // [NC][n] tangent moments and H Mdot
    void *rows;               // [n][n_theta] T: per-neighborhood gradient contributions
    int n_theta;
};
// Optional timing of library kernels with HIP events (see mtp_profile_enable).
void prof_mark(const char *name, bool begin, hipStream_t st);
struct ProfScope {
    const char *name;
    hipStream_t st;
    ProfScope(const char *n, hipStream_t s) : name(n), st(s) { prof_mark(name, true, st); }
    ~ProfScope() { prof_mark(name, false, st); }
};

}  // namespace mtp
