// Reductions and helpers of the evaluation path: force gather, per
// configuration energy / stress sums, row copies, preselection compaction.
#include <hip/hip_runtime.h>

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
// image of l).  FG_LANES lanes per atom, a fixed shuffle tree at the end, no
// atomics: results are bitwise reproducible.
constexpr int FG_LANES = 8;
template <typename T>
__global__ __launch_bounds__(256) void force_gather(int64_t n, int nt, int maxn, const int32_t *tcnt,
                                                    const int32_t *rev, const T *g, double *F) {
    const int sub = threadIdx.x % FG_LANES;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FG_LANES;
    const bool live = i < n;
    int tot = 0;
    if (live)
        for (int t = 0; t < nt; ++t) tot += tcnt[i * nt + t];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int p = sub; p < tot; p += FG_LANES) {
        const int64_t s = i * maxn + p;
        const int64_t q = rev[s];
        fx += double(g[3 * s]) - double(g[3 * q]);
        fy += double(g[3 * s + 1]) - double(g[3 * q + 1]);
        fz += double(g[3 * s + 2]) - double(g[3 * q + 2]);
    }
#pragma unroll
    for (int o = FG_LANES / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, 64);
        fy += __shfl_xor(fy, o, 64);
        fz += __shfl_xor(fz, o, 64);
    }
    if (live && sub == 0) {
        F[3 * i] = fx;
        F[3 * i + 1] = fy;
        F[3 * i + 2] = fz;
    }
}

// E_c = sum_i V_i and S_c = sum_i W_i over the atoms of configuration c
// (eq. 1) in FP64.  Block (c, s) sums every SUM_S-th chunk of 256 atoms of
// configuration c; the last block to finish adds the SUM_S partials of every
// configuration in order (deterministic).
constexpr int SUM_T = 256, SUM_S = 32;
__global__ __launch_bounds__(SUM_T) void cfg_sums(const int64_t *cfg_off, const double *site_e, const double *vir,
                                                  double *part, int n_cfg, double *energy, double *stress,
                                                  unsigned *ticket) {
    const int c = blockIdx.x / SUM_S, s = blockIdx.x % SUM_S;
    const int64_t b = cfg_off[c], e = cfg_off[c + 1];
    double acc[10];
    for (int k = 0; k < 10; ++k) acc[k] = 0.0;
    for (int64_t i = b + (int64_t)s * SUM_T + threadIdx.x; i < e; i += (int64_t)SUM_S * SUM_T) {
        if (site_e) acc[0] += site_e[i];
        if (vir)
            for (int k = 0; k < 9; ++k) acc[1 + k] += vir[9 * i + k];
    }
    __shared__ double sh[10][SUM_T];
    for (int k = 0; k < 10; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = SUM_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 10; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 10) part[(int64_t)blockIdx.x * 10 + threadIdx.x] = sh[threadIdx.x][0];
    if (!last_block(ticket)) return;
    for (int64_t t = threadIdx.x; t < (int64_t)n_cfg * 10; t += SUM_T) {
        const int cc = (int)(t / 10), k = (int)(t % 10);
        double v = 0.0;
        for (int q = 0; q < SUM_S; ++q) v += part[((int64_t)cc * SUM_S + q) * 10 + k];
        if (k == 0) {
            if (energy) energy[cc] = v;
        } else if (stress) {
            stress[9 * cc + k - 1] = v;
        }
    }
    reset_ticket(ticket);
}

template <typename T>
__global__ void copy_rows(const T *src, int ldb, int m, int64_t n, T *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * m) return;
    const int64_t r = i / m, c = i % m;
    dst[i] = src[r * ldb + c];
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

template <bool SCANNED>
__global__ __launch_bounds__(GRADE_ROWS) void select_write(const double *g, int64_t n, double thr,
                                                           const int32_t *blk, int32_t *idx, int32_t cap,
                                                           int32_t *count) {
    const int lane = threadIdx.x;
    int64_t off = 0;
    if (SCANNED) {
        off = blk[blockIdx.x];
    } else {
        for (int64_t b = lane; b < blockIdx.x; b += GRADE_ROWS) off += blk[b];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) off += __shfl_xor(off, d, 64);
    }
    const int64_t i = (int64_t)blockIdx.x * GRADE_ROWS + lane;
    const bool flag = i < n && g[i] > thr;
    const unsigned long long sel = __ballot(flag);
    const int64_t pos = off + __popcll(sel & ((1ull << lane) - 1ull));
    if (flag && pos < cap) idx[pos] = (int32_t)i;
    if (blockIdx.x == gridDim.x - 1 && lane == 0) {
        const int64_t tot = off + __popcll(sel);
        *count = (int32_t)(tot < cap ? tot : cap);
    }
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

void launch_zero(void *p, size_t bytes, hipStream_t st) {
    const size_t w = (bytes + 3) / 4;
    if (!w) return;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((w + 255) / 256)), dim3(256), 0, st, static_cast<uint32_t *>(p), w);
}

void launch_force_gather(const mtp_nbrs *nb, const void *gbuf, int precision, double *forces, hipStream_t st) {
    const int64_t n = nb->n_atoms;
    if (!n) return;
    const dim3 grid((unsigned)((n * FG_LANES + 255) / 256));
    if (precision == MTP_FP64)
        hipLaunchKernelGGL(force_gather<double>, grid, dim3(256), 0, st, n, nb->n_types, nb->max_nbrs,
                           nb->tcnt.as<int32_t>(), nb->rev.as<int32_t>(), static_cast<const double *>(gbuf), forces);
    else
        hipLaunchKernelGGL(force_gather<float>, grid, dim3(256), 0, st, n, nb->n_types, nb->max_nbrs,
                           nb->tcnt.as<int32_t>(), nb->rev.as<int32_t>(), static_cast<const float *>(gbuf), forces);
}

void launch_cfg_sums(const mtp_system *s, const double *site_e, const double *virial, double *energy, double *stress,
                     hipStream_t st, DevBuf &work, unsigned *ticket) {
    if (s->n_cfg <= 0) return;
    work.ensure(sizeof(double) * 10 * SUM_S * (size_t)s->n_cfg);
    hipLaunchKernelGGL(cfg_sums, dim3((unsigned)(s->n_cfg * SUM_S)), dim3(SUM_T), 0, st, s->cfg_off, site_e, virial,
                       work.as<double>(), s->n_cfg, energy, stress, ticket);
}

void launch_copy_rows(const void *src, int ldb, int m, int64_t n, int precision, void *dst, hipStream_t st) {
    const int64_t tot = n * m;
    if (!tot) return;
    const dim3 grid((unsigned)((tot + 255) / 256));
    if (precision == MTP_FP64)
        hipLaunchKernelGGL(copy_rows<double>, grid, dim3(256), 0, st, static_cast<const double *>(src), ldb, m, n,
                           static_cast<double *>(dst));
    else
        hipLaunchKernelGGL(copy_rows<float>, grid, dim3(256), 0, st, static_cast<const float *>(src), ldb, m, n,
                           static_cast<float *>(dst));
}

void launch_select_write(const double *gamma, int64_t n, double thr, int32_t *blk, int32_t *idx, int32_t cap,
                         int32_t *count, hipStream_t st) {
    if (n == 0) {
        launch_zero(count, sizeof(int32_t), st);
        return;
    }
    const int64_t nb = (n + GRADE_ROWS - 1) / GRADE_ROWS;
    if (nb <= SEL_DIRECT_BLOCKS) {
        hipLaunchKernelGGL(select_write<false>, dim3((unsigned)nb), dim3(GRADE_ROWS), 0, st, gamma, n, thr, blk, idx,
                           cap, count);
    } else {
        hipLaunchKernelGGL(select_scan, dim3(1), dim3(SCAN_T), 0, st, blk, nb);
        hipLaunchKernelGGL(select_write<true>, dim3((unsigned)nb), dim3(GRADE_ROWS), 0, st, gamma, n, thr, blk, idx,
                           cap, count);
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
