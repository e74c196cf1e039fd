// Reductions and helpers of the evaluation path: force gather, per
// configuration energy / stress sums, row copies, preselection compaction.
#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "internal.hpp"

namespace mtp {
namespace {

__global__ void zero_kernel(uint32_t *p, size_t n_words) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_words) p[i] = 0u;
}

// F_l = sum_{p in list(l)} (g_p - g_rev(p)): the first sum is -dV_l/dx_l, the
// second collects dV_i/dx_l over every neighborhood i that holds l (or an
// image of l).  The pair kernel wrote the first sum per atom into F and each
// g_p at the slot rev(p), so the second is the sum over l's own slots:
// F_l -= sum_{p in list(l)} h_p.  FG_LANES lanes per atom, a fixed shuffle
// tree at the end, no atomics: results are bitwise reproducible.  A block
// holds SUM_CHUNK atoms; with `part` it also writes that chunk's partial
// energy / virial sums.
constexpr int FG_LANES = 8;
static_assert(256 / FG_LANES == SUM_CHUNK, "one force_gather block per sum chunk");
template <typename T>
__device__ inline void gather_block(int64_t blk, int64_t n, int nt, int maxn, const int32_t *tcnt, const T *h,
                                    double *F) {
    const int sub = threadIdx.x % FG_LANES;
    const int64_t i = (blk * 256 + threadIdx.x) / FG_LANES;   // blocks of 256 threads
    const bool live = i < n;
    const int64_t ic = live ? i : 0;
    int tot = 0;
#pragma unroll
    for (int t = 0; t < MAX_TYPES; ++t) tot += t < nt ? tcnt[ic * nt + t] : 0;
    if (!live) tot = 0;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    // FG_DEPTH pairs per lane at a time, every load unconditional so that they
    // are all in flight together: a slot past the count reads the atom's
    // last slot (in bounds) and adds nothing.  FG_LANES x FG_DEPTH = 40 pairs
    // in one round covers a dense crystal's neighborhood at R_cut = 5 A
    // (33 pairs) without a second memory round
    constexpr int FG_DEPTH = 5;
    const T *hi = h + ic * (int64_t)maxn * 3;
    for (int p0 = sub; p0 < tot; p0 += FG_DEPTH * FG_LANES) {
        T hq[FG_DEPTH][3];
#pragma unroll
        for (int d = 0; d < FG_DEPTH; ++d) {
            const int p = p0 + d * FG_LANES < maxn ? p0 + d * FG_LANES : maxn - 1;
#pragma unroll
            for (int k = 0; k < 3; ++k) hq[d][k] = hi[3 * p + k];
        }
#pragma unroll
        for (int d = 0; d < FG_DEPTH; ++d) {
            if (p0 + d * FG_LANES < tot) {
                fx += double(hq[d][0]);
                fy += double(hq[d][1]);
                fz += double(hq[d][2]);
            }
        }
    }
#pragma unroll
    for (int o = FG_LANES / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, 64);
        fy += __shfl_xor(fy, o, 64);
        fz += __shfl_xor(fz, o, 64);
    }
    if (live && sub == 0) {
        F[3 * i] -= fx;
        F[3 * i + 1] -= fy;
        F[3 * i + 2] -= fz;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void force_gather(int64_t n, int nt, int maxn, const int32_t *tcnt, const T *g,
                                                    double *F, const double *site_e, const double *vir, double *part) {
    gather_block<T>(blockIdx.x, n, nt, maxn, tcnt, g, F);
    if (part) chunk_partials(blockIdx.x, n, site_e, vir, part);   // uniform branch
}

// the chunk partials alone (energy or stress without forces)
__global__ __launch_bounds__(256) void cfg_partials(int64_t n, const double *site_e, const double *vir,
                                                    double *part) {
    chunk_partials(blockIdx.x, n, site_e, vir, part);
}

// E_c = sum_i V_i and S_c = sum_i W_i over the atoms [b, e) of configuration
// c (eq. 1), one block per configuration: the partials of the chunks that
// lie inside [b, e), plus the atoms of the chunks it shares with its
// neighbors.  Fixed assignment of terms to threads and a fixed reduction
// tree: deterministic.
__device__ inline void cfg_final_block(int c, const int64_t *cfg_off, const double *site_e, const double *vir,
                                       const double *part, double *energy, double *stress) {
    __shared__ double sp[4][10];
    const int64_t b = cfg_off[c], e = cfg_off[c + 1];
    const int64_t cb = (b + SUM_CHUNK - 1) / SUM_CHUNK, ce = e / SUM_CHUNK;   // whole chunks [cb, ce)
    double acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.0;
    auto atom = [&](int64_t i) {
        if (site_e) acc[0] += site_e[i];
        if (vir)
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[1 + k] += vir[9 * i + k];
    };
    if (cb < ce) {
        for (int64_t k = cb + threadIdx.x; k < ce; k += 256)
#pragma unroll
            for (int q = 0; q < 10; ++q) acc[q] += part[k * 10 + q];
        for (int64_t i = b + threadIdx.x; i < cb * SUM_CHUNK; i += 256) atom(i);
        for (int64_t i = ce * SUM_CHUNK + threadIdx.x; i < e; i += 256) atom(i);
    } else {
        for (int64_t i = b + threadIdx.x; i < e; i += 256) atom(i);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 10; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 10; ++q) sp[w][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < 10) {
        const int t = threadIdx.x;
        const double v = ((sp[0][t] + sp[1][t]) + sp[2][t]) + sp[3][t];
        if (t == 0) {
            if (energy) energy[c] = v;
        } else if (stress) {
            stress[9 * c + t - 1] = v;
        }
    }
}

__global__ __launch_bounds__(256) void cfg_final(const int64_t *cfg_off, const double *site_e, const double *vir,
                                                 const double *part, double *energy, double *stress) {
    cfg_final_block(blockIdx.x, cfg_off, site_e, vir, part, energy, stress);
}

// Configuration-mode rows b(cfg) = sum_i b_i over the atoms of each
// configuration, in FP64, in two steps like the energy sums: partial sums
// over chunks of ROW_CHUNK atoms (thread t of a block adds column t, t + 256,
// ... of its chunk's rows in atom order), then one block per configuration
// adds the partials of its whole chunks and the rows of the chunks it shares
// with its neighbors.  Fixed order throughout.  Rows and results are
// column-major (entry (i, k) at rows[k * n + i]).
constexpr int ROW_CHUNK = 64;
__global__ __launch_bounds__(256) void row_partials(const double *rows, int ldb, int64_t n, double *part) {
    const int64_t a0 = (int64_t)blockIdx.x * ROW_CHUNK;
    const int64_t a1 = a0 + ROW_CHUNK < n ? a0 + ROW_CHUNK : n;
    for (int k = threadIdx.x; k < ldb; k += 256) {
        const double *col = rows + (int64_t)k * n;
        double acc = 0.0;
        for (int64_t i = a0; i < a1; ++i) acc += col[i];
        part[(int64_t)blockIdx.x * ldb + k] = acc;
    }
}

__global__ __launch_bounds__(256) void row_final(const double *rows, int ldb, int64_t n, const double *part,
                                                 const int64_t *cfg_off, int n_cfg, double *out) {
    const int c = blockIdx.x;
    const int64_t b = cfg_off[c], e = cfg_off[c + 1];
    const int64_t cb = (b + ROW_CHUNK - 1) / ROW_CHUNK, ce = e / ROW_CHUNK;   // whole chunks [cb, ce)
    for (int k = threadIdx.x; k < ldb; k += 256) {
        const double *col = rows + (int64_t)k * n;
        double acc = 0.0;
        if (cb < ce) {
            for (int64_t i = b; i < cb * ROW_CHUNK; ++i) acc += col[i];
            for (int64_t q = cb; q < ce; ++q) acc += part[q * ldb + k];
            for (int64_t i = ce * ROW_CHUNK; i < e; ++i) acc += col[i];
        } else {
            for (int64_t i = b; i < e; ++i) acc += col[i];
        }
        out[(int64_t)k * n_cfg + c] = acc;
    }
}

// ---- extrapolation-controlled runs ---------------------------------------
// Largest value of g[0..n) and its lowest index (one block).
constexpr int AMAX_T = 1024;
__global__ __launch_bounds__(AMAX_T) void argmax_kernel(const double *g, int64_t n, double *best, int32_t *where) {
    __shared__ double sv[AMAX_T];
    __shared__ int64_t si[AMAX_T];
    double bv = -HUGE_VAL;
    int64_t bi = n;
    for (int64_t i = threadIdx.x; i < n; i += AMAX_T) {
        const double v = g[i];
        if (v > bv) {   // strided ascending: the first of equal values is kept
            bv = v;
            bi = i;
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = AMAX_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double ov = sv[threadIdx.x + w];
            const int64_t oi = si[threadIdx.x + w];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (best) *best = sv[0];
        if (where) *where = (int32_t)si[0];
    }
}

// Candidates of the spherical fragment: atom j = t / S and image shift number
// s = t % S.  The shift counts from the image of j nearest to the center c
// (per periodic axis the rounded fractional offset w), so n = n' - w with
// n' in [-K, K] per axis; key = cutoff^2 - |x_j + n H - x_c|^2 (> 0 inside).
struct CutGeom {
    double H[9], Hinv[9];   // rows: lattice vectors; Hinv: inverse of H
    int K[3];               // shift range per axis (0 on non-periodic axes)
    int per[3];
};
__device__ inline void cut_candidate(const CutGeom &G, const double *pos, int64_t j, int c, int64_t s, double r[3],
                                     int n[3]) {
    const double d[3] = {pos[3 * j] - pos[3 * c], pos[3 * j + 1] - pos[3 * c + 1], pos[3 * j + 2] - pos[3 * c + 2]};
    const int w3 = 2 * G.K[2] + 1, w2 = 2 * G.K[1] + 1;
    const int np[3] = {(int)(s / (w2 * w3)) - G.K[0], (int)((s / w3) % w2) - G.K[1], (int)(s % w3) - G.K[2]};
    for (int k = 0; k < 3; ++k) {
        const double f = d[0] * G.Hinv[k] + d[1] * G.Hinv[3 + k] + d[2] * G.Hinv[6 + k];   // fractional offset
        const int w = G.per[k] ? (int)rint(f) : 0;
        n[k] = np[k] - w;
    }
    for (int a = 0; a < 3; ++a) r[a] = d[a] + n[0] * G.H[a] + n[1] * G.H[3 + a] + n[2] * G.H[6 + a];
}

__global__ void cut_keys(int64_t n, int64_t S, CutGeom G, const double *pos, const int32_t *center, double cutoff,
                         double *keys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * S) return;
    double r[3];
    int sh[3];
    cut_candidate(G, pos, t / S, *center, t % S, r, sh);
    keys[t] = cutoff * cutoff - (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

__global__ void cut_gather(int64_t S, CutGeom G, const double *pos, const int32_t *type, const int32_t *center,
                           const int32_t *idx, const int32_t *count, double *pos_out, int32_t *type_out,
                           int32_t *src_out, int32_t *shift_out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= *count) return;
    const int64_t t = idx[k], j = t / S;
    const int c = *center;
    double r[3];
    int sh[3];
    cut_candidate(G, pos, j, c, t % S, r, sh);
    for (int a = 0; a < 3; ++a) {
        if (pos_out) pos_out[3 * k + a] = pos[3 * j + a] + sh[0] * G.H[a] + sh[1] * G.H[3 + a] + sh[2] * G.H[6 + a];
        if (shift_out) shift_out[3 * k + a] = sh[a];
    }
    if (type_out) type_out[k] = type[j];
    if (src_out) src_out[k] = (int32_t)j;
}

// velocity Verlet: v += h F / m (h = dt / 2 times the unit factor), then x += dt v
__global__ void md_kick_drift(int64_t n, double *x, double *v, const double *F, const int32_t *type,
                              const double *inv_m, double h, double dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double im = inv_m[type[i]];
    for (int a = 0; a < 3; ++a) {
        const double vi = v[3 * i + a] + h * F[3 * i + a] * im;
        v[3 * i + a] = vi;
        x[3 * i + a] += dt * vi;
    }
}

__global__ void md_kick(int64_t n, double *v, const double *F, const int32_t *type, const double *inv_m, double h) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double im = inv_m[type[i]];
    for (int a = 0; a < 3; ++a) v[3 * i + a] += h * F[3 * i + a] * im;
}

// Residual terms of eq. 7 for one kind of target: g = 2 w (y - t) (the
// upstream gradient dL/dy) and, per block of 256 entries, the partial sum of
// w (y - t)^2 (added in a fixed tree).
__global__ __launch_bounds__(256) void fit_residual(int64_t n, const double *y, const double *t, double w, double *g,
                                                    double *part) {
    __shared__ double sp[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double r = 0.0;
    if (i < n) {
        r = y[i] - t[i];
        g[i] = 2.0 * w * r;
    }
    sp[threadIdx.x] = w * r * r;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sp[threadIdx.x] += sp[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sp[0];
}

// FIRE relaxation: out = {F.v, F.F, v.v, max_i |F_i|^2} over all atoms (one
// block, fixed reduction order), and the velocity mixing v <- a v + b F.
constexpr int FIRE_T = 1024;
__global__ __launch_bounds__(FIRE_T) void fire_norms(int64_t n, const double *F, const double *v, double *out) {
    __shared__ double s[4][FIRE_T];
    double p = 0.0, ff = 0.0, vv = 0.0, fm = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += FIRE_T) {
        double fi = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double f = F[3 * i + a], u = v[3 * i + a];
            p += f * u;
            fi += f * f;
            vv += u * u;
        }
        ff += fi;
        fm = fmax(fm, fi);
    }
    s[0][threadIdx.x] = p;
    s[1][threadIdx.x] = ff;
    s[2][threadIdx.x] = vv;
    s[3][threadIdx.x] = fm;
    __syncthreads();
    for (int w = FIRE_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
            s[2][threadIdx.x] += s[2][threadIdx.x + w];
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

__global__ void fire_mix(int64_t n3, double *v, const double *F, double a, double b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) v[i] = a * v[i] + b * F[i];
}

// column-major rows -> row-major [n][m] (through a 32 x 32 LDS tile: both
// the reads and the writes are consecutive words)
__global__ __launch_bounds__(256) void copy_rows(const double *src, int64_t ldn, int m, int64_t n, double *dst) {
    __shared__ double t[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    const int c0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int q = ty; q < 32; q += 8) {
        const int c = c0 + q;
        const int64_t r = r0 + tx;
        t[q][tx] = (c < m && r < n) ? src[(int64_t)c * ldn + r] : 0.0;
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + q;
        const int c = c0 + tx;
        if (r < n && c < m) dst[r * m + c] = t[tx][q];
    }
}

// Preselection: indices with gamma > thr in ascending order.  Blocks of
// GRADE_ROWS rows (one wavefront): select_count writes each block's count
// (the grade kernels can write the same counts themselves); select_write
// gives block b the offset sum_{b' < b} count[b'] by summing the counts
// before it (no cross-block synchronisation), ranks its rows by a ballot and
// writes them; the block holding the last row writes the total (clamped to
// the capacity).
__global__ __launch_bounds__(GRADE_ROWS) void select_count(const double *g, int64_t n, double thr, int32_t *blk) {
    const int64_t i = (int64_t)blockIdx.x * GRADE_ROWS + threadIdx.x;
    const unsigned long long sel = __ballot(i < n && g[i] > thr);
    if (threadIdx.x == 0) blk[blockIdx.x] = __popcll(sel);
}

// Above SEL_DIRECT_BLOCKS blocks the summing would grow quadratically:
// select_scan (one block) first turns the counts into exclusive offsets, in
// place, with the total in blk[nb], and select_write reads its offset.
constexpr int64_t SEL_DIRECT_BLOCKS = 1024;
constexpr int SCAN_T = 1024;
__global__ __launch_bounds__(SCAN_T) void select_scan(int32_t *blk, int64_t nb) {
    __shared__ int32_t s[SCAN_T];
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_T) {
        const int64_t k = base + threadIdx.x;
        const int32_t x = k < nb ? blk[k] : 0;
        const int32_t inc = block_scan<SCAN_T>(x, s);
        if (k < nb) blk[k] = carry + inc - x;
        carry += s[SCAN_T - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[nb] = carry;
}

// one wavefront places the selected rows of preselection block gb (of nb);
// blk holds `per` counts per block of GRADE_ROWS rows (one per grade block)
template <bool SCANNED>
__device__ inline void select_write_wave(int64_t gb, int64_t nb, const double *g, int64_t n, double thr,
                                         const int32_t *blk, int per, int32_t *idx, int32_t cap, int32_t *count) {
    const int lane = threadIdx.x & 63;
    int64_t off = 0;
    if (SCANNED) {
        off = blk[gb * per];
    } else {
        for (int64_t b = lane; b < gb * per; b += GRADE_ROWS) off += blk[b];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) off += __shfl_xor(off, d, 64);
    }
    const int64_t i = gb * GRADE_ROWS + lane;
    const bool flag = i < n && g[i] > thr;
    const unsigned long long sel = __ballot(flag);
    const int64_t pos = off + __popcll(sel & ((1ull << lane) - 1ull));
    if (flag && pos < cap) idx[pos] = (int32_t)i;
    if (gb == nb - 1 && lane == 0) {
        const int64_t tot = off + __popcll(sel);
        *count = (int32_t)(tot < cap ? tot : cap);
    }
}

// four preselection blocks per block of 256 threads; with n_cfg > 0 the
// first n_cfg blocks add the configuration sums instead (one launch for both
// at the end of the evaluation)
// blocks [0, n_cfg): configuration sums; [n_cfg, n_cfg + ga.blocks): the
// force gather (GatherArgs; it waits for nothing the grade writes, and its
// own launch would cost more than its blocks); the rest: one wavefront per
// GRADE_ROWS rows of the preselection.
template <bool SCANNED>
__global__ __launch_bounds__(256) void select_write(const double *g, int64_t n, double thr, const int32_t *blk,
                                                    int per, int32_t *idx, int32_t cap, int32_t *count, int n_cfg,
                                                    const int64_t *cfg_off, const double *site_e, const double *vir,
                                                    const double *part, double *energy, double *stress,
                                                    const GatherArgs ga) {
    if ((int)blockIdx.x < n_cfg) {
        cfg_final_block(blockIdx.x, cfg_off, site_e, vir, part, energy, stress);
        return;
    }
    const int64_t b = (int64_t)blockIdx.x - n_cfg;
    if (b < ga.blocks) {
        if (ga.precision == MTP_FP64)
            gather_block<double>(b, ga.n, ga.nt, ga.maxn, ga.tcnt, static_cast<const double *>(ga.g), ga.F);
        else
            gather_block<float>(b, ga.n, ga.nt, ga.maxn, ga.tcnt, static_cast<const float *>(ga.g), ga.F);
        return;
    }
    const int64_t nb = (n + GRADE_ROWS - 1) / GRADE_ROWS;
    const int64_t gb = (b - ga.blocks) * 4 + (threadIdx.x >> 6);
    if (gb < nb) select_write_wave<SCANNED>(gb, nb, g, n, thr, blk, per, idx, cap, count);
}

// column sums of the per-neighborhood gradient rows, FP64, fixed order:
// block (column tile, atom chunk) -> partial; then partials in chunk order
constexpr int CS_CH = 64;
template <typename T>
__global__ __launch_bounds__(256) void col_partial(const T *rows, int64_t n, int ncol, double *part) {
    const int col = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
    const int64_t chunk = (n + CS_CH - 1) / CS_CH;
    const int64_t i0 = (int64_t)blockIdx.y * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    double s = 0.0;
    if (col < ncol)
        for (int64_t i = i0 + g; i < i1; i += 4) s += double(rows[i * ncol + col]);
    __shared__ double sh[4][64];
    sh[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && col < ncol)
        part[(int64_t)blockIdx.y * ncol + col] = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) +
                                                 sh[3][threadIdx.x];
}

__global__ void col_final(const double *part, int ncol, double *out) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncol) return;
    double s = 0.0;
    for (int ch = 0; ch < CS_CH; ++ch) s += part[(int64_t)ch * ncol + col];
    out[col] = s;
}

}  // namespace

void launch_column_sums(const void *rows, int precision, int64_t n, int ncol, double *out, hipStream_t st,
                        DevBuf &work) {
    work.ensure(sizeof(double) * CS_CH * (size_t)ncol);
    const dim3 grid((unsigned)((ncol + 63) / 64), CS_CH);
    if (precision == MTP_FP64)
        hipLaunchKernelGGL(col_partial<double>, grid, dim3(256), 0, st, static_cast<const double *>(rows), n, ncol,
                           work.as<double>());
    else
        hipLaunchKernelGGL(col_partial<float>, grid, dim3(256), 0, st, static_cast<const float *>(rows), n, ncol,
                           work.as<double>());
    hipLaunchKernelGGL(col_final, dim3((unsigned)((ncol + 255) / 256)), dim3(256), 0, st, work.as<double>(), ncol, out);
}

// Scratch of mtp_energy_forces_stress_noalloc: a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends).
// Host code never uses the array's name as an address (on the host it is a
// stand-in, not device memory): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

void *noalloc_scratch(int device) {
    static std::mutex mu;
    static void *ptr[64] = {};
    MTP_CHECK(device >= 0 && device < 64, MTP_E_INVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        void *p = nullptr;
        MTP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MTP_CHECK(p != nullptr, MTP_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        ptr[device] = p;
    }
    return ptr[device];
}

void launch_zero(void *p, size_t bytes, hipStream_t st) {
    const size_t w = (bytes + 3) / 4;
    if (!w) return;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((w + 255) / 256)), dim3(256), 0, st, static_cast<uint32_t *>(p), w);
}

void launch_force_gather(const mtp_nbrs *nb, const void *gbuf, int precision, double *forces, hipStream_t st,
                         const double *site_e, const double *virial, double *part) {
    const int64_t n = nb->n_atoms;
    if (!n) return;
    const dim3 grid((unsigned)((n * FG_LANES + 255) / 256));
    if (precision == MTP_FP64)
        hipLaunchKernelGGL(force_gather<double>, grid, dim3(256), 0, st, n, nb->n_types, nb->max_nbrs,
                           nb->tcnt.as<int32_t>(), static_cast<const double *>(gbuf), forces, site_e, virial, part);
    else
        hipLaunchKernelGGL(force_gather<float>, grid, dim3(256), 0, st, n, nb->n_types, nb->max_nbrs,
                           nb->tcnt.as<int32_t>(), static_cast<const float *>(gbuf), forces, site_e, virial, part);
}

size_t cfg_partials_bytes(int64_t n) {
    return sizeof(double) * 10 * (size_t)std::max<int64_t>(1, (n + SUM_CHUNK - 1) / SUM_CHUNK);
}

void launch_cfg_partials(int64_t n, const double *site_e, const double *virial, double *part, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(cfg_partials, dim3((unsigned)((n + SUM_CHUNK - 1) / SUM_CHUNK)), dim3(256), 0, st, n,
                           site_e, virial, part);
}

void launch_cfg_final(const mtp_system *s, const double *site_e, const double *virial, const double *part,
                      double *energy, double *stress, hipStream_t st) {
    if (s->n_cfg <= 0) return;
    hipLaunchKernelGGL(cfg_final, dim3((unsigned)s->n_cfg), dim3(256), 0, st, s->cfg_off, site_e, virial, part,
                       energy, stress);
}

void launch_copy_rows(const double *src, int64_t ldn, int m, int64_t n, double *dst, hipStream_t st) {
    if (n == 0 || m == 0) return;
    const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
    hipLaunchKernelGGL(copy_rows, grid, dim3(256), 0, st, src, ldn, m, n, dst);
}

size_t cfg_row_partials_bytes(int64_t n, int ldb) {
    return sizeof(double) * (size_t)ldb * (size_t)std::max<int64_t>(1, (n + ROW_CHUNK - 1) / ROW_CHUNK);
}

void launch_cfg_rows(const double *rows, int ldb, int64_t n, const mtp_system *s, double *part, double *out,
                     hipStream_t st) {
    if (s->n_cfg <= 0) return;
    const unsigned nch = (unsigned)((n + ROW_CHUNK - 1) / ROW_CHUNK);
    if (nch) hipLaunchKernelGGL(row_partials, dim3(nch), dim3(256), 0, st, rows, ldb, n, part);
    hipLaunchKernelGGL(row_final, dim3((unsigned)s->n_cfg), dim3(256), 0, st, rows, ldb, n, part, s->cfg_off,
                       s->n_cfg, out);
}

void launch_argmax(const double *g, int64_t n, double *best, int32_t *where, hipStream_t st) {
    hipLaunchKernelGGL(argmax_kernel, dim3(1), dim3(AMAX_T), 0, st, g, n, best, where);
}

void launch_md_step(int half, int64_t n, double *x, double *v, const double *F, const int32_t *type,
                    const double *inv_m, double h, double dt, hipStream_t st) {
    if (n == 0) return;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (half == 0)
        hipLaunchKernelGGL(md_kick_drift, grid, dim3(256), 0, st, n, x, v, F, type, inv_m, h, dt);
    else
        hipLaunchKernelGGL(md_kick, grid, dim3(256), 0, st, n, v, F, type, inv_m, h);
}

int64_t cut_fragment(const double *pos, const int32_t *type, int64_t n, const double *H, const int *per,
                     const double *g, double cutoff, int32_t cap, double *pos_out, int32_t *type_out,
                     int32_t *src_out, int32_t *shift_out, int32_t *count_dev, int32_t *center_dev, hipStream_t st,
                     DevBuf &keys, DevBuf &idx, DevBuf &work) {
    CutGeom G{};
    for (int k = 0; k < 9; ++k) G.H[k] = H[k];
    const double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                       H[2] * (H[3] * H[7] - H[4] * H[6]);
    MTP_CHECK(std::fabs(det) > 1e-12, MTP_E_INVAL, "the cell matrix is singular");
    // inverse by cofactors (Hinv[r][c] = cof(c, r) / det)
    G.Hinv[0] = (H[4] * H[8] - H[5] * H[7]) / det;
    G.Hinv[1] = (H[2] * H[7] - H[1] * H[8]) / det;
    G.Hinv[2] = (H[1] * H[5] - H[2] * H[4]) / det;
    G.Hinv[3] = (H[5] * H[6] - H[3] * H[8]) / det;
    G.Hinv[4] = (H[0] * H[8] - H[2] * H[6]) / det;
    G.Hinv[5] = (H[2] * H[3] - H[0] * H[5]) / det;
    G.Hinv[6] = (H[3] * H[7] - H[4] * H[6]) / det;
    G.Hinv[7] = (H[1] * H[6] - H[0] * H[7]) / det;
    G.Hinv[8] = (H[0] * H[4] - H[1] * H[3]) / det;
    int64_t S = 1;
    for (int k = 0; k < 3; ++k) {
        // height of the cell along axis k: volume / |a_l x a_m|
        const double *a = H + 3 * ((k + 1) % 3), *b = H + 3 * ((k + 2) % 3);
        const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
        const double h = std::fabs(det) / std::sqrt(cx * cx + cy * cy + cz * cz);
        G.per[k] = per[k];
        G.K[k] = per[k] ? (int)std::floor(cutoff / h + 0.5) + 1 : 0;
        MTP_CHECK(G.K[k] <= 64, MTP_E_INVAL, "the cutoff spans more than 64 cells");
        S *= 2 * G.K[k] + 1;
    }
    const int64_t tot = n * S;
    MTP_CHECK(tot < ((int64_t)1 << 31), MTP_E_INVAL, "atoms x image shifts must stay below 2^31");
    keys.ensure(sizeof(double) * (size_t)tot);
    idx.ensure(sizeof(int32_t) * (size_t)std::max<int32_t>(cap, 1));
    launch_argmax(g, n, nullptr, center_dev, st);
    hipLaunchKernelGGL(cut_keys, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, S, G, pos, center_dev,
                       cutoff, keys.as<double>());
    launch_select(keys.as<double>(), tot, 0.0, idx.as<int32_t>(), cap, count_dev, st, work);
    if (cap > 0)
        hipLaunchKernelGGL(cut_gather, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, st, S, G, pos, type,
                           center_dev, idx.as<int32_t>(), count_dev, pos_out, type_out, src_out, shift_out);
    return tot;
}

int64_t launch_fit_residual(int64_t n, const double *y, const double *t, double w, double *g, double *part,
                            hipStream_t st) {
    const int64_t nb = (n + 255) / 256;
    if (nb) hipLaunchKernelGGL(fit_residual, dim3((unsigned)nb), dim3(256), 0, st, n, y, t, w, g, part);
    return nb;
}

void launch_fire_norms(int64_t n, const double *F, const double *v, double *out, hipStream_t st) {
    hipLaunchKernelGGL(fire_norms, dim3(1), dim3(FIRE_T), 0, st, n, F, v, out);
}

void launch_fire_mix(int64_t n, double *v, const double *F, double a, double b, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(fire_mix, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, st, 3 * n, v, F, a, b);
}

GatherArgs gather_args(const mtp_nbrs *nb, const void *gbuf, int precision, double *forces) {
    GatherArgs ga{};
    ga.n = nb->n_atoms;
    ga.nt = nb->n_types;
    ga.maxn = nb->max_nbrs;
    ga.tcnt = nb->tcnt.as<int32_t>();
    ga.g = gbuf;
    ga.precision = precision;
    ga.F = forces;
    ga.blocks = (ga.n * FG_LANES + 255) / 256;
    return ga;
}

void launch_select_write(const double *gamma, int64_t n, double thr, int32_t *blk, int32_t *idx, int32_t cap,
                         int32_t *count, hipStream_t st, const CfgSums *sums, const GatherArgs *gather,
                         int count_rows) {
    MTP_CHECK(count_rows > 0 && GRADE_ROWS % count_rows == 0, MTP_E_INVAL, "preselection count granularity");
    const int per = GRADE_ROWS / count_rows;
    const GatherArgs ga = gather ? *gather : GatherArgs{};
    const int n_cfg = sums ? sums->s->n_cfg : 0;
    const int64_t *off = sums ? sums->s->cfg_off : nullptr;
    const double *se = sums ? sums->site_e : nullptr, *vir = sums ? sums->virial : nullptr;
    const double *part = sums ? sums->part : nullptr;
    double *energy = sums ? sums->energy : nullptr, *stress = sums ? sums->stress : nullptr;
    if (n == 0) {
        launch_zero(count, sizeof(int32_t), st);
        if (sums) launch_cfg_final(sums->s, se, vir, part, energy, stress, st);
        return;
    }
    const int64_t nb = (n + GRADE_ROWS - 1) / GRADE_ROWS;
    const int64_t ncount = (n + count_rows - 1) / count_rows;   // entries of blk
    const dim3 grid((unsigned)(n_cfg + ga.blocks + (nb + 3) / 4));
    if (ncount <= SEL_DIRECT_BLOCKS) {
        hipLaunchKernelGGL(select_write<false>, grid, dim3(256), 0, st, gamma, n, thr, blk, per, idx, cap, count, n_cfg,
                           off, se, vir, part, energy, stress, ga);
    } else {
        // exclusive offsets in place: entry gb * per is where block gb starts
        hipLaunchKernelGGL(select_scan, dim3(1), dim3(SCAN_T), 0, st, blk, ncount);
        hipLaunchKernelGGL(select_write<true>, grid, dim3(256), 0, st, gamma, n, thr, blk, per, idx, cap, count, n_cfg,
                           off, se, vir, part, energy, stress, ga);
    }
}

void launch_select(const double *gamma, int64_t n, double thr, int32_t *idx, int32_t cap, int32_t *count,
                   hipStream_t st, DevBuf &work) {
    const int64_t nb = (n + GRADE_ROWS - 1) / GRADE_ROWS;
    work.ensure(sizeof(int32_t) * (size_t)(nb + 1));
    if (n > 0)
        hipLaunchKernelGGL(select_count, dim3((unsigned)nb), dim3(GRADE_ROWS), 0, st, gamma, n, thr,
                           work.as<int32_t>());
    launch_select_write(gamma, n, thr, work.as<int32_t>(), idx, cap, count, st);
}

}  // namespace mtp
