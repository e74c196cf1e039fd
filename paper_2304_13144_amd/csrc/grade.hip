// Extrapolation grades and the active set (MLIP-3 paper Sec. II.C-D).
//
//   gamma_i = max_p |(b_i A^-1)_p|, argmax p (lowest index on ties)
//
// The rows b (FP64 in both forms) are column-major: entry (i, k) at
// brow[k * ldn + i].
//
// FP64 form: v_mfma_f64_16x16x4 tiles.  A block of 512 threads owns 64 rows
// of C; each wavefront 16 rows and half of each pass of 224 columns.  The
// block keeps a running max / argmax per row, so C is never written.  A^-1
// (<= m^2 x 8 B) stays L2-resident.
//
// Mixed form: an int8 slice product with exact int32 accumulation (the
// scheme of Ozaki et al. for accurate matrix products from low-precision
// units).  Columns are equilibrated by powers of two, D_k = 2^-round(log2
// max_i |A_ik|), so that b D and D^-1 A^-1 have entries of like size; each
// row of b D and each column of D^-1 A^-1 is scaled by a power of two into
// (-1, 1) and cut into NSL signed 7-bit digits (round to nearest: the first
// digit of x 2^6, then of the remainder times 2^7), so x = 2^e sum_t d_t
// 2^-(6 + 7t) up to 2^-(6 + 7 NSL) of the row (column) maximum.  Products of
// digits of levels s + t <= NSL are summed on v_mfma_i32_16x16x64_i8 with no
// rounding at all (|sum| < 2^31), and C = 2^(e_i + f_c) sum_q acc_q
// 2^-(12 + 7q) in FP64.  FP32 rows or FP32 accumulation cannot hold gamma
// to 1e-5 on the level-16 alloy's active set (column-equilibrated
// condition number ~2e5, cancellation in b A^-1 of ~4e3); this product
// keeps ~34 bits of each operand and rounds nothing until the final FP64
// sum.
//
// Also here: A^-1 by Gauss-Jordan elimination (FP64, partial pivoting) and
// the MaxVol swap loop with Sherman-Morrison updates (FP64 only).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace mtp {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));   // (HIP's double2 is a struct: arrays of it end up in scratch)

__device__ inline void better(double v, int c, double &bv, int &bc) {
    if (v > bv || (v == bv && c < bc)) {
        bv = v;
        bc = c;
    }
}

// Result layouts of the two MFMAs (16x16 tile, lane l, register r):
//   f64 16x16x4:      row (l/16) + 4 r, column l % 16
//   i32 16x16x64 i8:  row 4 (l/16) + r, column l % 16

// FP64: a block of eight wavefronts owns 64 rows; wave w takes rows
// 16 (w % 4) .. + 16 and one half (w / 4) of each pass of CT = 32 HALF
// columns (HALF MFMA column blocks, accumulators in registers).  k runs in
// chunks of 16 through three LDS buffers, fetched two chunks ahead: chunk
// c + 2 is in flight from global memory into registers while the MFMAs
// consume chunk c, and chunk c + 1 (fetched one iteration earlier) is stored
// to its buffer -- one barrier per chunk, a full chunk of MFMA work to cover
// each load.  Two wavefronts per SIMD keep the matrix pipe busy across the
// barrier.  The two column halves of a row meet in LDS at the end.
//
// The inner loop has no branches: loads read clamped addresses (row n - 1
// for rows past n, whose results are never written; k rows of A^-1 past m
// meet the zero padding of the b rows, columns past m are never compared)
// and every wave runs all HALF column blocks, so the compiler can interleave
// the LDS reads of the next MFMAs with the current ones.  HALF is chosen per
// m on the host (the smallest padding of m to passes of 32 HALF columns).
constexpr int GF_ROWS = 64, GF_KC = 16, GF_NBUF = 3;
template <int HALF>
__global__ __launch_bounds__(512) void grade_f64_wide(const double *__restrict__ brow, int64_t ldn, int64_t n,
                                                 const double *__restrict__ Ainv, int m, double *gamma,
                                                 int32_t *argmax, double thr, int32_t *sel_blk) {
    constexpr int CT = 32 * HALF;
    // B rows padded by 16 doubles: the four k rows one MFMA operand read
    // touches then start 32 banks apart instead of on the same bank
    constexpr int CTP = CT + 16;
    __shared__ double sA[GF_NBUF][GF_ROWS][GF_KC + 1];
    __shared__ double sB[GF_NBUF][GF_KC][CTP];
    __shared__ double s_best[2][GF_ROWS];
    __shared__ int s_idx[2][GF_ROWS];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rg = wave & 3, half = wave >> 2;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * GF_ROWS;
    const int nchunk = (m + GF_KC - 1) / GF_KC;
    double best[4] = {-1.0, -1.0, -1.0, -1.0};
    int bidx[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    constexpr int RA = GF_ROWS * GF_KC / 512, RB = GF_KC * CT / 512;
    static_assert(RA * 512 == GF_ROWS * GF_KC && RB * 512 == GF_KC * CT, "staging must tile the block");
    struct Regs {
        double a[RA], b[RB];
    };
    for (int ct0 = 0; ct0 < m; ct0 += CT) {
        const int cb0 = half * HALF;
        doublex4 acc[HALF];
#pragma unroll
        for (int c = 0; c < HALF; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
        auto fetch = [&](Regs &R, int ch) {
            const int k0 = ch * GF_KC;
#pragma unroll
            for (int q = 0; q < RA; ++q) {   // 64 consecutive rows of one column per wavefront
                const int e = tid + 512 * q;
                const int r = e % GF_ROWS, k = k0 + e / GF_ROWS;   // k < ldb: the rows are padded with zeros
                R.a[q] = brow[(int64_t)k * ldn + min(row0 + r, n - 1)];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int e = tid + 512 * q;
                const int k = k0 + e / CT, c = ct0 + e % CT;
                R.b[q] = Ainv[(int64_t)min(k, m - 1) * m + min(c, m - 1)];
            }
        };
        auto store = [&](const Regs &R, int buf) {
#pragma unroll
            for (int q = 0; q < RA; ++q) {
                const int e = tid + 512 * q;
                sA[buf][e % GF_ROWS][e / GF_ROWS] = R.a[q];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int e = tid + 512 * q;
                sB[buf][e / CT][e % CT] = R.b[q];
            }
        };
        auto compute = [&](int buf) {
#pragma unroll
            for (int kk = 0; kk < GF_KC; kk += 4) {
                const double av = sA[buf][rg * 16 + lr][kk + lk];
#pragma unroll
                for (int c = 0; c < HALF; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sB[buf][kk + lk][(cb0 + c) * 16 + lr],
                                                                  acc[c], 0, 0, 0);
            }
        };
        // one iteration: fetch chunk ch + 2 into F, compute chunk ch, store chunk ch + 1 (held in S)
        auto step = [&](int ch, Regs &F, const Regs &S) {
            if (ch + 2 < nchunk) fetch(F, ch + 2);
            compute(ch % GF_NBUF);
            if (ch + 1 < nchunk) store(S, (ch + 1) % GF_NBUF);
            __syncthreads();
        };
        Regs R0, R1;
        __syncthreads();   // the previous pass no longer reads the buffers
        fetch(R0, 0);
        if (nchunk > 1) fetch(R1, 1);
        store(R0, 0);
        __syncthreads();
        for (int ch = 0; ch < nchunk; ch += 2) {
            step(ch, R0, R1);   // R0 (chunk ch, stored) is free: chunk ch + 2 goes there
            if (ch + 1 < nchunk) step(ch + 1, R1, R0);
        }
#pragma unroll
        for (int c = 0; c < HALF; ++c) {
            const int col = ct0 + (cb0 + c) * 16 + lr;
            if (col < m)
#pragma unroll
                for (int r = 0; r < 4; ++r) better(fabs(acc[c][r]), col, best[r], bidx[r]);
        }
    }
    // the 16 lanes of a row, then the two column halves
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double ov = __shfl_xor(best[r], o, 64);
            const int oc = __shfl_xor(bidx[r], o, 64);
            better(ov, oc, best[r], bidx[r]);
        }
    if (lr == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s_best[half][rg * 16 + lk + 4 * r] = best[r];
            s_idx[half][rg * 16 + lk + 4 * r] = bidx[r];
        }
    __syncthreads();
    if (tid < GF_ROWS) {   // wavefront 0: one row per lane
        double bv = s_best[0][tid];
        int bc = s_idx[0][tid];
        better(s_best[1][tid], s_idx[1][tid], bv, bc);
        const bool live = row0 + tid < n;
        if (live) {
            gamma[row0 + tid] = bv;
            if (argmax) argmax[row0 + tid] = bc;
        }
        // preselection counts (gamma > thr) of this block, for select_write
        const unsigned long long sel = __ballot(live && bv > thr);
        if (sel_blk && tid == 0) sel_blk[blockIdx.x] = __popcll(sel);
    }
}

// FP64, m <= 32 GR_NK_MAX (288): a block of 512 threads = 64 rows x two halves of
// the column tiles (wavefront w: row group w % 4, half w / 4, tiles h, h + 2,
// ...), so that every SIMD runs two wavefronts.  A wavefront holds its 16 rows
// in registers for the whole product in the MFMA operand layout (lane l: row
// l % 16, k = 4 s + l / 16 of k step s; 8 NK steps of four).  A^-1 is stored
// column tile by column tile in the order the lanes read it ([tile][s][lane]:
// k = 4 s + l / 16, column 16 tile + l % 16, zero past m), so each half stages
// its tile into LDS as one contiguous copy (double-buffered, the next tile's
// loads in flight during the MFMAs, one barrier per tile) and a wavefront
// reads its operand with one 8-byte LDS read per k step.  The k steps go
// round-robin to four accumulators (four independent MFMA chains), added at
// the end of the tile; the two halves' maxima meet in LDS at the end.
constexpr int GR_NK_MAX = 9;   // 32-k chunks: m <= 288 (two halves x two buffers of a tile in LDS)
template <int NK>
__global__ __launch_bounds__(512) void grade_f64(const double *__restrict__ brow, int64_t ldn, int64_t n,
                                                 const double *__restrict__ L, int m, double *gamma,
                                                 int32_t *argmax, double thr, int32_t *sel_blk) {
    constexpr int KS = 8 * NK;                 // k steps of four
    constexpr int TILE = KS * 64;              // doubles of one column tile
    constexpr int PER = TILE / 2 / 256;        // 16-byte pieces per thread of a half (NK)
    static_assert(PER * 512 == TILE, "tile staging");
    __shared__ doublex2 sB[2][2][TILE / 2];    // [half][buffer]
    __shared__ double s_best[2][GF_ROWS];
    __shared__ int s_idx[2][GF_ROWS];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rg = wave & 3, half = wave >> 2, ht = tid & 255;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * GF_ROWS + rg * 16;
    const int ntile = (m + 15) / 16;
    const int nstep = (ntile + 1) / 2;         // tiles per half, rounded up (both halves pass every barrier)
    doublex2 pre[PER];
    auto fetch = [&](int tile) {
        tile = tile < ntile ? tile : ntile - 1;   // past the last tile: an in-bounds tile, never compared
        const doublex2 *src = reinterpret_cast<const doublex2 *>(L + (int64_t)tile * TILE);
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = src[ht + 256 * q];
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) sB[half][buf][ht + 256 * q] = pre[q];
    };
    fetch(half);
    // this lane's row, k = 4 s + lk (the rows are zero past m up to ldb >= 32 NK)
    double a[KS];
    {
        const double *bp = brow + min(row0 + lr, n - 1) + (int64_t)lk * ldn;   // rows past n: clamped, never written
#pragma unroll
        for (int s = 0; s < KS; ++s) a[s] = bp[(int64_t)(4 * s) * ldn];
    }
    double best[4] = {-1.0, -1.0, -1.0, -1.0};
    int bidx[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    stash(0);
    // the rows are waited for here, once: with their loads still counted at
    // the loop's entry, every tile's products would also wait for the next
    // tile's prefetch (the load counter is in order), exposing its latency
#pragma unroll
    for (int s = 0; s < KS; ++s) __asm__ volatile("" ::"v"(a[s]));
    __syncthreads();
    for (int st = 0; st < nstep; ++st) {
        const int buf = st & 1, tile = 2 * st + half;
        if (st + 1 < nstep) fetch(tile + 2);
        doublex4 acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
        const double *b = reinterpret_cast<const double *>(sB[half][buf]) + lane;
#pragma unroll
        for (int s = 0; s < KS; s += 4)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s + c], b[64 * (s + c)], acc[c], 0, 0, 0);
        const int col = 16 * tile + lr;
        if (col < m)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                better(fabs((acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r])), col, best[r], bidx[r]);
        if (st + 1 < nstep) stash(buf ^ 1);
        __syncthreads();
    }
    // the 16 lanes of a row (columns), then the two halves
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double ov = __shfl_xor(best[r], o, 64);
            const int oc = __shfl_xor(bidx[r], o, 64);
            better(ov, oc, best[r], bidx[r]);
        }
    if (lr == 0)   // f64 layout: lane l, register r -> row l / 16 + 4 r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s_best[half][rg * 16 + lk + 4 * r] = best[r];
            s_idx[half][rg * 16 + lk + 4 * r] = bidx[r];
        }
    __syncthreads();
    if (tid < GF_ROWS) {   // wavefront 0: one row per lane
        double bv = s_best[0][tid];
        int bc = s_idx[0][tid];
        better(s_best[1][tid], s_idx[1][tid], bv, bc);
        const int64_t row = (int64_t)blockIdx.x * GF_ROWS + tid;
        const bool live = row < n;
        if (live) {
            gamma[row] = bv;
            if (argmax) argmax[row] = bc;
        }
        const unsigned long long sel = __ballot(live && bv > thr);
        if (sel_blk && tid == 0) sel_blk[blockIdx.x] = __popcll(sel);
    }
}

// The same product in blocks of 256 threads = 32 rows x two halves of the
// column tiles, one LDS buffer per half (57 KB at m = 212), so that two
// blocks share a CU: one block's barriers, tile staging and epilogues then
// overlap the other's MFMAs (with one block per CU every wavefront of the CU
// meets the same barrier at the same time, and the MFMA units idle through
// it).  Per tile: barrier (every wavefront has read the buffer), the next
// tile's pieces from registers into LDS, barrier, the next-but-one tile's
// loads issued, the products.  Counts of gamma > thr per 32 rows.
constexpr int GF2_ROWS = 32;
template <int NK>
__global__ __launch_bounds__(256, 2) void grade_f64_pair(const double *__restrict__ brow, int64_t ldn, int64_t n,
                                                         const double *__restrict__ L, int m, double *gamma,
                                                         int32_t *argmax, double thr, int32_t *sel_blk) {
    constexpr int KS = 8 * NK;                 // k steps of four
    constexpr int TILE = KS * 64;              // doubles of one column tile
    constexpr int PER = TILE / 2 / 128;        // 16-byte pieces per thread of a half
    static_assert(PER * 256 == TILE, "tile staging");
    __shared__ doublex2 sB[2][TILE / 2];       // [half]
    __shared__ double s_best[2][GF2_ROWS];
    __shared__ int s_idx[2][GF2_ROWS];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rg = wave & 1, half = wave >> 1, ht = tid & 127;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * GF2_ROWS + rg * 16;
    const int ntile = (m + 15) / 16;
    const int nstep = (ntile + 1) / 2;         // tiles per half, rounded up (both halves pass every barrier)
    doublex2 pre[PER];
    auto fetch = [&](int tile) {               // unconditional: past the last tile, an in-bounds tile
        tile = tile < ntile ? tile : ntile - 1;
        const doublex2 *src = reinterpret_cast<const doublex2 *>(L + (int64_t)tile * TILE);
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = src[ht + 128 * q];
    };
    fetch(half);
    double a[KS];
    {
        const double *bp = brow + min(row0 + lr, n - 1) + (int64_t)lk * ldn;   // rows past n: clamped, never written
#pragma unroll
        for (int s = 0; s < KS; ++s) a[s] = bp[(int64_t)(4 * s) * ldn];
    }
    double best[4] = {-1.0, -1.0, -1.0, -1.0};
    int bidx[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    for (int st = 0; st < nstep; ++st) {
        const int tile = 2 * st + half;
        __syncthreads();   // every wavefront has read the buffer (and, at st = 0, nothing has)
#pragma unroll
        for (int q = 0; q < PER; ++q) sB[half][ht + 128 * q] = pre[q];
        __syncthreads();
        fetch(tile + 2);
        doublex4 acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
        const double *b = reinterpret_cast<const double *>(sB[half]) + lane;
#pragma unroll
        for (int s = 0; s < KS; s += 4)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s + c], b[64 * (s + c)], acc[c], 0, 0, 0);
        const int col = 16 * tile + lr;
        if (col < m)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                better(fabs((acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r])), col, best[r], bidx[r]);
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double ov = __shfl_xor(best[r], o, 64);
            const int oc = __shfl_xor(bidx[r], o, 64);
            better(ov, oc, best[r], bidx[r]);
        }
    if (lr == 0)   // f64 layout: lane l, register r -> row l / 16 + 4 r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s_best[half][rg * 16 + lk + 4 * r] = best[r];
            s_idx[half][rg * 16 + lk + 4 * r] = bidx[r];
        }
    __syncthreads();
    if (tid < 64) {   // wavefront 0: one row per lane (32 rows)
        const int q = tid < GF2_ROWS ? tid : 0;
        double bv = s_best[0][q];
        int bc = s_idx[0][q];
        better(s_best[1][q], s_idx[1][q], bv, bc);
        const int64_t row = (int64_t)blockIdx.x * GF2_ROWS + tid;
        const bool live = tid < GF2_ROWS && row < n;
        if (live) {
            gamma[row] = bv;
            if (argmax) argmax[row] = bc;
        }
        const unsigned long long sel = __ballot(live && bv > thr);
        if (sel_blk && tid == 0) sel_blk[blockIdx.x] = __popcll(sel);
    }
}

// FP64 with k outermost: a block of 512 threads owns 64 rows (row group w %
// 4 of wavefront w, half w / 4 of the column tiles: tiles h NK .. h NK + NK -
// 1).  A wavefront keeps the accumulators of all NK of its tiles (8 NK
// registers) and runs k in chunks of KC k steps: per chunk, KC values of its
// rows (loaded two chunks ahead) times the chunk's operands of its NK tiles,
// KC NK independent MFMAs.  The rows are never held whole, so their loads
// spread over the product instead of all arriving before the first MFMA.
// Each half's chunk of A^-1 (NK pieces of KC x 512 bytes, one per tile, in
// the lane order of f64_stage_ainv) is loaded DIST chunks ahead into
// registers and stored to LDS one chunk ahead, double-buffered: one barrier
// per chunk.  The 64 rows of a block share every staged chunk, so A^-1
// crosses from L2 once per 64 rows.  The chunk loop is unrolled in full
// (2 NK x 4 / KC chunks), so every wait count is exact.  KC = 8, DIST = 1:
// 112 KB of LDS at m = 224, one block per CU (the fewest barriers, for
// launches of about one block per CU); KC = 2, DIST = 2: 28 KB and fewer
// registers, two blocks per CU (for larger launches).
template <int NK, int KC, int DIST>
__global__ __launch_bounds__(512) void grade_f64_kouter(const double *__restrict__ brow, int64_t ldn, int64_t n,
                                                        const double *__restrict__ L, int m, double *gamma,
                                                        int32_t *argmax, double thr, int32_t *sel_blk) {
    constexpr int KS = 8 * NK;                 // k steps of four
    constexpr int NCH = KS / KC;               // chunks
    static_assert(NCH * KC == KS, "chunks tile the k steps");
    constexpr int CH = KC * NK * 64;           // doubles of one half's chunk in LDS: [step][tile][lane]
    constexpr int PIECES = NK * KC * 32;       // its 16-byte pieces: [tile][step][32]
    constexpr int PER = (PIECES + 255) / 256;  // per thread of the half
    __shared__ double sB[2][2][CH];            // [half][buffer]
    __shared__ double s_best[2][GF_ROWS];
    __shared__ int s_idx[2][GF_ROWS];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rg = wave & 3, half = wave >> 2, ht = tid & 255;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * GF_ROWS + rg * 16;
    const int ntile = (m + 15) / 16;
    // k steps that reach a column below m: the later ones multiply the rows'
    // zero padding, and are skipped (m > 32 (NK - 1), so every step up to
    // 8 (NK - 1) is needed and the test folds away for all but the last few)
    const int ksn = (m + 3) / 4;
    doublex2 pre[DIST][PER];
    auto fetch = [&](int c) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = ht + 256 * q;
            if (PIECES % 256 == 0 || e < PIECES) {
                const int j = e / (KC * 32), p = e % (KC * 32);
                const int t = min(half * NK + j, ntile - 1);   // past the last tile: an in-bounds tile, never compared
                pre[c % DIST][q] = reinterpret_cast<const doublex2 *>(L + ((int64_t)t * KS + KC * c) * 64)[p];
            }
        }
    };
    auto stash = [&](int buf, int c) {   // piece p of tile j: step p / 32, lanes 2 (p % 32) and 2 (p % 32) + 1
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = ht + 256 * q;
            if (PIECES % 256 == 0 || e < PIECES) {
                const int j = e / (KC * 32), p = e % (KC * 32);
                *reinterpret_cast<doublex2 *>(&sB[half][buf][((p >> 5) * NK + j) * 64 + 2 * (p & 31)]) =
                    pre[c % DIST][q];
            }
        }
    };
    // this lane's row at k = 4 s + lk (zero past m up to ldb >= 32 NK); rows past n: clamped, never written
    const double *bp = brow + min(row0 + lr, n - 1) + (int64_t)lk * ldn;
    double a[NCH][KC];
    auto load_rows = [&](int c) {
#pragma unroll
        for (int s = 0; s < KC; ++s) a[c][s] = bp[(int64_t)(4 * (KC * c + s)) * ldn];
    };
    fetch(0);
    load_rows(0);
    if (NCH > 1) load_rows(1);
    stash(0, 0);
#pragma unroll
    for (int d = 1; d <= DIST; ++d)
        if (d < NCH) fetch(d);
    __syncthreads();
    double best[4] = {-1.0, -1.0, -1.0, -1.0};
    int bidx[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    doublex4 acc[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) acc[j] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (c + 2 < NCH) load_rows(c + 2);
        const double *b = sB[half][c & 1] + lane;
#pragma unroll
        for (int s = 0; s < KC; ++s)
            if (KC * c + s <= 8 * (NK - 1) || KC * c + s < ksn)   // uniform
#pragma unroll
                for (int j = 0; j < NK; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][s], b[(s * NK + j) * 64], acc[j], 0, 0, 0);
        if (c + 1 < NCH) {
            stash((c + 1) & 1, c + 1);   // its last readers passed the previous barrier
            if (c + 1 + DIST < NCH) fetch(c + 1 + DIST);
            __syncthreads();
        }
    }
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int col = 16 * (half * NK + j) + lr;
        if (col < m)
#pragma unroll
            for (int r = 0; r < 4; ++r) better(fabs(acc[j][r]), col, best[r], bidx[r]);
    }
    // the 16 lanes of a row (columns), then the two halves
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double ov = __shfl_xor(best[r], o, 64);
            const int oc = __shfl_xor(bidx[r], o, 64);
            better(ov, oc, best[r], bidx[r]);
        }
    if (lr == 0)   // f64 layout: lane l, register r -> row l / 16 + 4 r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s_best[half][rg * 16 + lk + 4 * r] = best[r];
            s_idx[half][rg * 16 + lk + 4 * r] = bidx[r];
        }
    __syncthreads();
    if (tid < GF_ROWS) {   // wavefront 0: one row per lane
        double bv = s_best[0][tid];
        int bc = s_idx[0][tid];
        better(s_best[1][tid], s_idx[1][tid], bv, bc);
        const int64_t row = (int64_t)blockIdx.x * GF_ROWS + tid;
        const bool live = row < n;
        if (live) {
            gamma[row] = bv;
            if (argmax) argmax[row] = bc;
        }
        const unsigned long long sel = __ballot(live && bv > thr);
        if (sel_blk && tid == 0) sel_blk[blockIdx.x] = __popcll(sel);
    }
}

// A^-1 in the lane order of grade_f64: out[(tile * 8 NK + s) * 64 + l] =
// A^-1[4 s + l / 16][16 tile + l % 16], zero past m
__global__ void f64_stage_ainv(const double *Ainv, int m, int NK, int ntile, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)ntile * 8 * NK * 64;
    if (e >= tot) return;
    const int l = (int)(e % 64);
    const int64_t ts = e / 64;
    const int s = (int)(ts % (8 * NK)), tile = (int)(ts / (8 * NK));
    const int k = 4 * s + l / 16, c = 16 * tile + l % 16;
    out[e] = (k < m && c < m) ? Ainv[(int64_t)k * m + c] : 0.0;
}

// ---- mixed form: int8 slice product ----------------------------------------
// Block of 512 threads = 64 rows x two halves of the column tiles (wavefront
// w: row group w % 4, half w / 4, tiles h, h + 2, ...: two wavefronts per
// SIMD).  Each wavefront cuts its rows into digits and keeps them in
// registers in the MFMA operand layout (lane l: row l % 16, k = 64 s + 16 (l / 16) .. + 16 of k step
// s; KS steps, m <= 64 KS).  The digits of D^-1 A^-1 are stored tile by tile
// in exactly the order the lanes read them ([tile][s][slice][lane][16]), so
// each half stages its column tile into LDS as one contiguous copy (five
// 16-byte loads per thread at KS = 4), double-buffered, one barrier per
// tile, and every wavefront reads its operand with one 16-byte LDS read per
// slice and k step; the halves' maxima meet in LDS at the end.  Result layout of the 16x16 i32 tile: row 4 (l / 16) +
// r, column l % 16.
constexpr int GI_SL = 5;                  // digits per operand
constexpr int GI_LEV = GI_SL + 1;         // levels s + t = 0 .. GI_SL summed
constexpr int GI_KS_MAX = 5;              // k steps of 64 held in registers: m <= 320
constexpr int GI_ROWS = 64;               // rows per block (and per preselection count)
typedef int i32x4 __attribute__((ext_vector_type(4)));

template <int KS>
__global__ __launch_bounds__(512) void grade_i8(const double *__restrict__ brow, int ldb, int64_t ldn, int64_t n,
                                                const i32x4 *__restrict__ S, const int32_t *__restrict__ fexp,
                                                const double *__restrict__ dsc, int m, int CP, double *gamma,
                                                int32_t *argmax, double thr, int32_t *sel_blk) {
    constexpr int TILE = KS * GI_SL * 64;     // 16-byte pieces of one column tile
    constexpr int PER = (TILE + 255) / 256;   // pieces per thread of a half
    // one LDS area: first the rows' digits [row group][s][slice][lane], then
    // the column tiles [half][buffer][TILE] (the same size)
    __shared__ i32x4 sm[4 * TILE];
    __shared__ double s_mx[2][GI_ROWS];
    __shared__ double s_best[2][GI_ROWS];
    __shared__ int s_idx[2][GI_ROWS];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rg = wave & 3, half = wave >> 2, ht = tid & 255;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * GI_ROWS + rg * 16;
    const int64_t arow = min(row0 + lr, n - 1);   // rows past n: clamped, never written
    const double *bp = brow + arow;
    const int ntile = (m + 15) / 16;
    const int nstep = (ntile + 1) / 2;   // tiles per half, rounded up (both halves pass every barrier)
    // the first column tile's digits in flight while the rows are cut
    i32x4 pre[PER];
    auto fetch = [&](int tile) {
        tile = tile < ntile ? tile : ntile - 1;   // past the last tile: an in-bounds tile, never compared
        const i32x4 *src = S + (int64_t)tile * TILE;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = ht + 256 * q;
            if (TILE % 256 == 0 || e < TILE) pre[q] = src[e];
        }
    };
    auto stash = [&](int buf) {
        i32x4 *dst = sm + (2 * half + buf) * TILE;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = ht + 256 * q;
            if (TILE % 256 == 0 || e < TILE) dst[e] = pre[q];
        }
    };
    fetch(half);
    // the two halves' wavefronts of a row group cut it together: k steps
    // s = half, half + 2, ...  All of this wavefront's values of b D are
    // loaded in one batch (one memory latency, not one per group of loads);
    // the rows have ldb >= 64 KS columns, zero past m, and D_k = 0 past m
    constexpr int NH = (KS + 1) / 2;   // k steps per half (the second half has one less for odd KS)
    double x[NH][16];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int s = half + 2 * i;
        const int k0 = 64 * (s < KS ? s : KS - 1) + 16 * lk;   // a step past KS: read again, not used
        const double *p = bp + (int64_t)k0 * ldn;
#pragma unroll
        for (int j = 0; j < 16; j += 4) {
            const double4 d = *reinterpret_cast<const double4 *>(dsc + k0 + j);
            x[i][j] = p[(int64_t)j * ldn] * d.x;
            x[i][j + 1] = p[(int64_t)(j + 1) * ldn] * d.y;
            x[i][j + 2] = p[(int64_t)(j + 2) * ldn] * d.z;
            x[i][j + 3] = p[(int64_t)(j + 3) * ldn] * d.w;
        }
    }
    // the row's largest |b_k D_k|: this wavefront's steps, the four lanes of the
    // row, then the two halves
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < NH; ++i)
        if (half + 2 * i < KS)
#pragma unroll
            for (int j = 0; j < 16; ++j) mx = fmax(mx, fabs(x[i][j]));
    mx = fmax(mx, __shfl_xor(mx, 16, 64));
    mx = fmax(mx, __shfl_xor(mx, 32, 64));
    if (lane < 16) s_mx[half][rg * 16 + lane] = mx;
    __syncthreads();
    mx = fmax(s_mx[0][rg * 16 + lr], s_mx[1][rg * 16 + lr]);
    int erow;
    (void)frexp(mx, &erow);   // mx = f 2^erow, f in [0.5, 1); 0 for a zero row
    const double sc = ldexp(1.0, 6 - erow);
    // digits of this wavefront's k steps into LDS, one register per slice for each four k
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int s = half + 2 * i;
        if (s < KS)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned w[GI_SL] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    double r = x[i][4 * q + j] * sc;   // |r| < 64, exact
#pragma unroll
                    for (int t = 0; t < GI_SL; ++t) {
                        const double d = rint(r);
                        r = (r - d) * 128.0;
                        w[t] |= ((unsigned)(int)d & 0xffu) << (8 * j);
                    }
                }
                int *dig = reinterpret_cast<int *>(sm + ((rg * KS + s) * GI_SL) * 64 + lane) + q;
#pragma unroll
                for (int t = 0; t < GI_SL; ++t) dig[t * 64 * 4] = (int)w[t];
            }
    }
    __syncthreads();
    i32x4 A[GI_SL][KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int t = 0; t < GI_SL; ++t) A[t][s] = sm[((rg * KS + s) * GI_SL + t) * 64 + lane];
    // 2^(erow - 19) of the four result rows of this lane (row 4 lk + r is held by
    // lane 4 lk + r): level 1 (weight 2^-19) is the unit of the combined sums below
    double rsc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rsc[r] = ldexp(1.0, __shfl(erow, 4 * lk + r, 64) - 19);
    double best[4] = {-1.0, -1.0, -1.0, -1.0};
    int bidx[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    __syncthreads();   // every wavefront holds its digits: the area takes the column tiles
    stash(0);
    __syncthreads();
    for (int st = 0; st < nstep; ++st) {
        const int buf = st & 1, tile = 2 * st + half;
        // this tile's column scales before the next tile's prefetch: waiting
        // for them then leaves the prefetch in flight (the load counter is in
        // order, and the prefetch is issued on every path)
        const int col = 16 * tile + lr;
        const int fe = fexp[col < CP ? col : CP - 1];
        fetch(tile + 2);   // unconditional (clamped to a valid tile at the end), so that the wait count is known
        const i32x4 *sB = sm + (2 * half + buf) * TILE;
        i32x4 acc[GI_LEV];
#pragma unroll
        for (int q = 0; q < GI_LEV; ++q) acc[q] = i32x4{0, 0, 0, 0};
        // the operand of k step s + 1 is read from LDS while the MFMAs of step s run
        i32x4 B[2][GI_SL];
#pragma unroll
        for (int t = 0; t < GI_SL; ++t) B[0][t] = sB[t * 64 + lane];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s + 1 < KS)
#pragma unroll
                for (int t = 0; t < GI_SL; ++t) B[(s + 1) & 1][t] = sB[((s + 1) * GI_SL + t) * 64 + lane];
#pragma unroll
            for (int a = 0; a < GI_SL; ++a)
#pragma unroll
                for (int b = 0; a + b <= GI_SL && b < GI_SL; ++b)
                    acc[a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[a][s], B[s & 1][b], acc[a + b], 0, 0, 0);
        }
        const double cs = ldexp(1.0, fe);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // levels 0 + 1, 2 + 3, 4 + 5 exactly in int32 (|acc_q| < 2^23), then FP64:
            // C = 2^(erow + fexp - 19) (c01 + 2^-14 (c23 + 2^-14 c45))
            const int c01 = acc[0][r] * 128 + acc[1][r];
            const int c23 = acc[2][r] * 128 + acc[3][r];
            const int c45 = acc[4][r] * 128 + acc[5][r];
            const double v = fma(fma((double)c45, 0x1p-14, (double)c23), 0x1p-14, (double)c01);
            if (col < m) better(fabs(v * rsc[r] * cs), col, best[r], bidx[r]);
        }
        if (st + 1 < nstep) stash(buf ^ 1);
        __syncthreads();
    }
    // the 16 lanes of a row group (columns), then the two halves
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double ov = __shfl_xor(best[r], o, 64);
            const int oc = __shfl_xor(bidx[r], o, 64);
            better(ov, oc, best[r], bidx[r]);
        }
    if (lr == 0)   // i32 layout: lane l, register r -> row 4 (l / 16) + r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s_best[half][rg * 16 + 4 * lk + r] = best[r];
            s_idx[half][rg * 16 + 4 * lk + r] = bidx[r];
        }
    __syncthreads();
    if (tid < GI_ROWS) {   // wavefront 0: one row per lane
        double bv = s_best[0][tid];
        int bc = s_idx[0][tid];
        better(s_best[1][tid], s_idx[1][tid], bv, bc);
        const int64_t row = (int64_t)blockIdx.x * GI_ROWS + tid;
        const bool live = row < n;
        if (live) {
            gamma[row] = bv;
            if (argmax) argmax[row] = bc;
        }
        const unsigned long long sel = __ballot(live && bv > thr);
        if (sel_blk && tid == 0) sel_blk[blockIdx.x] = __popcll(sel);
    }
}

// D_k = 2^-round(log2 max_i |A_ik|) (0 past m, and for an all-zero column)
__global__ void i8_colscale(const double *A, int m, int KP, double *dsc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= KP) return;
    double mx = 0.0;
    if (k < m)
        for (int i = 0; i < m; ++i) mx = fmax(mx, fabs(A[(int64_t)i * m + k]));
    dsc[k] = mx > 0.0 ? ldexp(1.0, -(int)rint(log2(mx))) : 0.0;
}

// digits of column c of D^-1 A^-1, stored in the order the grade's lanes read
// them: [tile = c / 16][s = k / 64][slice][lane = c % 16 + 16 ((k % 64) / 16)][k % 16];
// one block per column (padded columns: zero)
__global__ __launch_bounds__(256) void i8_slice_ainv(const double *Ainv, int m, int KP, int CP, const double *dsc,
                                                     int8_t *S, int32_t *fexp) {
    __shared__ double sm[256];
    const int c = blockIdx.x;
    double mx = 0.0;
    for (int k = threadIdx.x; k < m; k += 256)
        if (c < m && dsc[k] > 0.0) mx = fmax(mx, fabs(Ainv[(int64_t)k * m + c] / dsc[k]));
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    int e;
    (void)frexp(sm[0], &e);
    if (threadIdx.x == 0) fexp[c] = e;
    const double sc = ldexp(1.0, 6 - e);
    const int KS = KP / 64;
    const int64_t tile_bytes = (int64_t)KS * GI_SL * 64 * 16;
    for (int k = threadIdx.x; k < KP; k += 256) {
        double r = (c < m && k < m && dsc[k] > 0.0) ? Ainv[(int64_t)k * m + c] / dsc[k] * sc : 0.0;
        const int s = k / 64, lane = c % 16 + 16 * ((k % 64) / 16);
        int8_t *dst = S + (c / 16) * tile_bytes + ((int64_t)(s * GI_SL) * 64 + lane) * 16 + k % 16;
        for (int t = 0; t < GI_SL; ++t) {
            const double d = rint(r);
            r = (r - d) * 128.0;
            dst[(int64_t)t * 64 * 16] = (int8_t)(int)d;
        }
    }
}

// ---- Gauss-Jordan inverse ---------------------------------------------------
// W = [A | I] (m x 2m, row-major) becomes [I | A^-1] by m elimination steps
// with partial pivoting (largest |W[r][c]| over r >= c, the lowest row on
// ties).  One launch per step c, one block per row r: every block finds the
// pivot p itself (the same search over column c in every block, so no
// grid-wide exchange is needed) and writes row r of the next W from the
// current one (two buffers: no block reads what another writes):
//   next[c] = cur[p] / cur[p][c]
//   next[p] = cur[c] - cur[c][c] next[c]          (p != c)
//   next[r] = cur[r] - cur[r][c] next[c]          (other rows)
// with column c set to the unit vector e_c exactly.  A pivot below 1e-300
// sets *singular, and every later step returns at once.
constexpr int GJ_T = 256;
__global__ __launch_bounds__(GJ_T) void gj_step(const double *__restrict__ cur, double *__restrict__ next, int m,
                                                int c, int32_t *singular) {
    __shared__ double sv[GJ_T / 64];
    __shared__ int si[GJ_T / 64];
    if (*singular) return;   // uniform: the flag was written by an earlier launch
    const int n2 = 2 * m, r = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double bv = -1.0;
    int bi = m;
    for (int q = c + tid; q < m; q += GJ_T) {
        const double v = fabs(cur[(int64_t)q * n2 + c]);
        if (v > bv) {   // rows visited in increasing order: the first maximum is kept
            bv = v;
            bi = q;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        sv[wave] = bv;
        si[wave] = bi;
    }
    __syncthreads();
    bv = sv[0];
    bi = si[0];
    for (int w = 1; w < GJ_T / 64; ++w)
        if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) {
            bv = sv[w];
            bi = si[w];
        }
    if (!(bv > 1e-300)) {
        if (r == 0 && tid == 0) *singular = 1;
        return;   // uniform over the block
    }
    const int p = bi;
    const double *prow = cur + (int64_t)p * n2;
    const double inv = 1.0 / prow[c];
    double *out = next + (int64_t)r * n2;
    if (r == c) {
        for (int k = tid; k < n2; k += GJ_T) out[k] = k == c ? 1.0 : prow[k] * inv;
        return;
    }
    const double *src = cur + (int64_t)(r == p ? c : r) * n2;
    const double f = src[c];
    for (int k = tid; k < n2; k += GJ_T) out[k] = k == c ? 0.0 : fma(-f, prow[k] * inv, src[k]);
}

__global__ void gj_setup(const double *A, int m, double *W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * 2 * m) return;
    const int r = (int)(e / (2 * m)), k = (int)(e % (2 * m));
    W[e] = k < m ? A[(int64_t)r * m + k] : (k - m == r ? 1.0 : 0.0);
}

__global__ void gj_extract(const double *W, int m, double *Ainv) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    const int r = (int)(e / m), k = (int)(e % m);
    Ainv[e] = W[(int64_t)r * 2 * m + m + k];
}

// ---- MaxVol (FP64) ----------------------------------------------------------
// C = cand * Ainv (plain FP64, one thread per entry)
__global__ void gemm_f64(const double *X, int64_t n, const double *Ainv, int m, double *C) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m;
    const int j = (int)(e % m);
    double s = 0.0;
    for (int k = 0; k < m; ++k) s = fma(X[i * m + k], Ainv[(int64_t)k * m + j], s);
    C[e] = s;
}

struct MVState {
    int32_t done, swaps, i, j;
    double piv;
};

constexpr int AM_T = 256;
__global__ void absmax_partial(const double *C, int64_t total, double *pv, int64_t *pi) {
    __shared__ double sv[AM_T];
    __shared__ int64_t si[AM_T];
    double bv = -1.0;
    int64_t bi = 0x7fffffffffffffffLL;
    for (int64_t e = (int64_t)blockIdx.x * AM_T + threadIdx.x; e < total; e += (int64_t)gridDim.x * AM_T) {
        const double v = fabs(C[e]);
        if (v > bv || (v == bv && e < bi)) {
            bv = v;
            bi = e;
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = AM_T / 2; w > 0; w >>= 1) {
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
        pv[blockIdx.x] = sv[0];
        pi[blockIdx.x] = si[0];
    }
}

__global__ void absmax_final(const double *pv, const int64_t *pi, int nb, int m, double thr, int max_swaps,
                             const double *C, MVState *st, int32_t *swap_cand, int32_t *swap_col) {
    if (threadIdx.x != 0) return;
    if (st->done) return;
    double bv = -1.0;
    int64_t bi = 0x7fffffffffffffffLL;
    for (int b = 0; b < nb; ++b)
        if (pv[b] > bv || (pv[b] == bv && pi[b] < bi)) {
            bv = pv[b];
            bi = pi[b];
        }
    if (!(bv > thr) || st->swaps >= max_swaps) {
        st->done = 1;
        return;
    }
    st->i = (int32_t)(bi / m);
    st->j = (int32_t)(bi % m);
    st->piv = C[bi];
    swap_cand[st->swaps] = st->i;
    swap_col[st->swaps] = st->j;
}

// save the pivot row of C and the pivot columns of C and A^-1
__global__ void mv_save(const double *C, int64_t n, const double *Ainv, int m, const MVState *st, double *crow,
                        double *ccol, double *acol) {
    if (st->done) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) {
        crow[t] = C[(int64_t)st->i * m + t];
        acol[t] = Ainv[t * m + st->j];
    }
    if (t < n) ccol[t] = C[t * m + st->j];
}

// C <- C - C[:,j] (c - e_j) / c_j; row i becomes the replaced row's coordinates
// e_j - (c - e_j) / c_j.  A^-1 <- A^-1 - A^-1[:,j] (c - e_j) / c_j.
__global__ void mv_update(double *C, int64_t n, double *Ainv, int m, const MVState *st, const double *crow,
                          const double *ccol, const double *acol) {
    if (st->done) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = st->j, i = st->i;
    const double pv = st->piv;
    if (e < n * m) {
        const int64_t r = e / m;
        const int k = (int)(e % m);
        const double v = (crow[k] - (k == j ? 1.0 : 0.0)) / pv;
        if (r == i) C[e] = (k == j ? 1.0 : 0.0) - v;
        else C[e] = C[e] - ccol[r] * v;
    }
    if (e < (int64_t)m * m) {
        const int64_t r = e / m;
        const int k = (int)(e % m);
        const double v = (crow[k] - (k == j ? 1.0 : 0.0)) / pv;
        Ainv[e] = Ainv[e] - acol[r] * v;
    }
}

// exchange the rows: A[j] <-> cand[i]
__global__ void mv_swap(double *A, double *cand, int m, MVState *st) {
    if (st->done) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) {
        const double t = A[(int64_t)st->j * m + k];
        A[(int64_t)st->j * m + k] = cand[(int64_t)st->i * m + k];
        cand[(int64_t)st->i * m + k] = t;
    }
}

__global__ void mv_count(MVState *st) {
    if (threadIdx.x == 0 && !st->done) st->swaps += 1;
}

__global__ void mv_init(MVState *st) {
    if (threadIdx.x == 0) {
        st->done = 0;
        st->swaps = 0;
        st->i = st->j = 0;
        st->piv = 0.0;
    }
}

}  // namespace

// digits of D^-1 A^-1 for the mixed product, after any change of A^-1
void prepare_split(ActiveSet &as, hipStream_t st) {
    const int m = as.m;
    as.KP8 = (m + 63) / 64 * 64;
    as.CP8 = (m + 15) / 16 * 16;
    as.s8.ensure((size_t)GI_SL * as.CP8 * as.KP8);
    as.fexp.ensure(sizeof(int32_t) * as.CP8);
    as.dsc.ensure(sizeof(double) * as.KP8);
    hipLaunchKernelGGL(i8_colscale, dim3((unsigned)((as.KP8 + 255) / 256)), dim3(256), 0, st, as.A.as<double>(), m,
                       as.KP8, as.dsc.as<double>());
    hipLaunchKernelGGL(i8_slice_ainv, dim3((unsigned)as.CP8), dim3(256), 0, st, as.Ainv.as<double>(), m, as.KP8,
                       as.CP8, as.dsc.as<double>(), as.s8.as<int8_t>(), as.fexp.as<int32_t>());
    if (m <= 32 * GR_NK_MAX) {   // A^-1 in the lane order of the FP64 product
        as.NK64 = (m + 31) / 32;
        const int ntile = (m + 15) / 16;
        const int64_t tot = (int64_t)ntile * 8 * as.NK64 * 64;
        as.lane64.ensure(sizeof(double) * (size_t)tot);
        hipLaunchKernelGGL(f64_stage_ainv, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, as.Ainv.as<double>(),
                           m, as.NK64, ntile, as.lane64.as<double>());
    }
}

bool slice_product_fits(int m) { return m <= 64 * GI_KS_MAX; }

// column blocks per wave (HALF): the pass width 32 HALF that pads m the
// least, the widest on ties
static int grade_half(int m) {
    int best = 7, pad = 1 << 30;
    for (int h = 7; h >= 1; --h) {
        const int w = 32 * h, p = (m + w - 1) / w * w;
        if (p < pad) {
            pad = p;
            best = h;
        }
    }
    return best;
}

template <int HALF>
static void launch_grade_f64_wide(const ActiveSet &as, const double *brow, int64_t ldn, int64_t n, double *gamma,
                                  int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk) {
    const dim3 grid((unsigned)((n + GF_ROWS - 1) / GF_ROWS));
    hipLaunchKernelGGL(grade_f64_wide<HALF>, grid, dim3(512), 0, st, brow, ldn, n, as.Ainv.as<double>(), as.m, gamma,
                       argmax, thr, sel_blk);
}

template <int NK>
static void launch_grade_f64(const ActiveSet &as, const double *brow, int64_t ldn, int64_t n, double *gamma,
                             int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk) {
    const dim3 grid((unsigned)((n + GF_ROWS - 1) / GF_ROWS));
    hipLaunchKernelGGL(grade_f64<NK>, grid, dim3(512), 0, st, brow, ldn, n, as.lane64.as<double>(), as.m, gamma,
                       argmax, thr, sel_blk);
}

template <int NK>
static void launch_grade_f64_pair(const ActiveSet &as, const double *brow, int64_t ldn, int64_t n, double *gamma,
                                  int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk) {
    const dim3 grid((unsigned)((n + GF2_ROWS - 1) / GF2_ROWS));
    hipLaunchKernelGGL(grade_f64_pair<NK>, grid, dim3(256), 0, st, brow, ldn, n, as.lane64.as<double>(), as.m, gamma,
                       argmax, thr, sel_blk);
}

template <int NK, int KC, int DIST>
static void launch_grade_f64_kouter(const ActiveSet &as, const double *brow, int64_t ldn, int64_t n, double *gamma,
                                    int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk) {
    const dim3 grid((unsigned)((n + GF_ROWS - 1) / GF_ROWS));
    hipLaunchKernelGGL((grade_f64_kouter<NK, KC, DIST>), grid, dim3(512), 0, st, brow, ldn, n, as.lane64.as<double>(),
                       as.m, gamma, argmax, thr, sel_blk);
}

template <int KS>
static void launch_grade_i8(const ActiveSet &as, const double *brow, int ldb, int64_t ldn, int64_t n, double *gamma,
                            int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk) {
    const dim3 grid((unsigned)((n + GI_ROWS - 1) / GI_ROWS));
    hipLaunchKernelGGL(grade_i8<KS>, grid, dim3(512), 0, st, brow, ldb, ldn, n, as.s8.as<i32x4>(),
                       as.fexp.as<int32_t>(), as.dsc.as<double>(), as.m, as.CP8, gamma, argmax, thr, sel_blk);
}

bool grade_sched_valid(const ActiveSet &as, int precision, int sched) {
    switch (sched) {
        case GRADE_AUTO: return true;
        case GRADE_F64_REG: return as.m <= 32 * GR_NK_MAX;
        case GRADE_F64_PAIR:
        case GRADE_F64_KOUTER:
        case GRADE_F64_KOUTER2: return as.m <= 32 * GR_NK_MAX;
        case GRADE_F64_LDS: return true;
        case GRADE_I8: return precision == MTP_MIXED && slice_product_fits(as.m);
        default: return false;
    }
}

static int grade_sched_resolve(const ActiveSet &as, int precision, int sched) {
    if (sched != GRADE_AUTO) return sched;
    if (precision == MTP_MIXED && slice_product_fits(as.m)) return GRADE_I8;
    return as.m <= 32 * GR_NK_MAX ? GRADE_F64_REG : GRADE_F64_LDS;
}

int grade_count_rows(const ActiveSet &as, int precision, int sched) {
    return grade_sched_resolve(as, precision, sched) == GRADE_F64_PAIR ? GF2_ROWS : GRADE_ROWS;
}

void launch_grade(const ActiveSet &as, int precision, const double *brow, int ldb, int64_t ldn, int64_t n,
                  double *gamma, int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk, int sched) {
    // every form counts the preselection per block of the same 64 rows
    static_assert(GRADE_ROWS == GF_ROWS && GRADE_ROWS == GI_ROWS, "preselection blocks are grade blocks");
    static_assert(GRADE_ROWS % GF2_ROWS == 0, "preselection blocks");
    MTP_CHECK(grade_sched_valid(as, precision, sched), MTP_E_INVAL, "grade: schedule not available for this m / precision");
    if (n == 0) return;
    MTP_CHECK(ldb >= (as.m + 31) / 32 * 32, MTP_E_INVAL, "grade: row length below the padded row length");
    MTP_CHECK(ldn >= n, MTP_E_INVAL, "grade: column stride below the row count");
    sched = grade_sched_resolve(as, precision, sched);
    if (sched == GRADE_I8) {
        MTP_CHECK(as.KP8 == (as.m + 63) / 64 * 64 && as.s8.ptr, MTP_E_INVAL, "grade: digits of A^-1 not prepared");
        MTP_CHECK(ldb >= as.KP8, MTP_E_INVAL, "grade: rows not padded to a multiple of 64 columns");
        switch (as.KP8 / 64) {
            case 1: launch_grade_i8<1>(as, brow, ldb, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 2: launch_grade_i8<2>(as, brow, ldb, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 3: launch_grade_i8<3>(as, brow, ldb, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 4: launch_grade_i8<4>(as, brow, ldb, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            default: launch_grade_i8<5>(as, brow, ldb, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        }
        return;
    }
    if (sched == GRADE_F64_KOUTER || sched == GRADE_F64_KOUTER2) {
        MTP_CHECK(as.NK64 == (as.m + 31) / 32 && as.lane64.ptr, MTP_E_INVAL, "grade: A^-1 not staged");
        MTP_CHECK(ldb >= 32 * as.NK64, MTP_E_INVAL, "grade: rows not padded to a multiple of 32 columns");
        const bool big = sched == GRADE_F64_KOUTER;   // eight k steps per chunk, else two, two chunks ahead
#define MTP_KOUTER_CASE(K)                                                                  \
    case K:                                                                                 \
        if (big)                                                                            \
            launch_grade_f64_kouter<K, 8, 1>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); \
        else                                                                                \
            launch_grade_f64_kouter<K, 2, 2>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); \
        break;
        switch (as.NK64) {
            MTP_KOUTER_CASE(1)
            MTP_KOUTER_CASE(2)
            MTP_KOUTER_CASE(3)
            MTP_KOUTER_CASE(4)
            MTP_KOUTER_CASE(5)
            MTP_KOUTER_CASE(6)
            MTP_KOUTER_CASE(7)
            MTP_KOUTER_CASE(8)
            default:
                MTP_KOUTER_CASE(9)
        }
#undef MTP_KOUTER_CASE
        return;
    }
    if (sched == GRADE_F64_PAIR) {
        MTP_CHECK(as.NK64 == (as.m + 31) / 32 && as.lane64.ptr, MTP_E_INVAL, "grade: A^-1 not staged");
        MTP_CHECK(ldb >= 32 * as.NK64, MTP_E_INVAL, "grade: rows not padded to a multiple of 32 columns");
        switch (as.NK64) {
            case 1: launch_grade_f64_pair<1>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 2: launch_grade_f64_pair<2>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 3: launch_grade_f64_pair<3>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 4: launch_grade_f64_pair<4>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 5: launch_grade_f64_pair<5>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 6: launch_grade_f64_pair<6>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 7: launch_grade_f64_pair<7>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 8: launch_grade_f64_pair<8>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            default: launch_grade_f64_pair<9>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        }
        return;
    }
    if (sched == GRADE_F64_REG) {
        MTP_CHECK(as.NK64 == (as.m + 31) / 32 && as.lane64.ptr, MTP_E_INVAL, "grade: A^-1 not staged");
        MTP_CHECK(ldb >= 32 * as.NK64, MTP_E_INVAL, "grade: rows not padded to a multiple of 32 columns");
        switch (as.NK64) {
            case 1: launch_grade_f64<1>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 2: launch_grade_f64<2>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 3: launch_grade_f64<3>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 4: launch_grade_f64<4>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 5: launch_grade_f64<5>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 6: launch_grade_f64<6>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 7: launch_grade_f64<7>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            case 8: launch_grade_f64<8>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
            default: launch_grade_f64<9>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        }
        return;
    }
    switch (grade_half(as.m)) {
        case 1: launch_grade_f64_wide<1>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        case 2: launch_grade_f64_wide<2>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        case 3: launch_grade_f64_wide<3>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        case 4: launch_grade_f64_wide<4>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        case 5: launch_grade_f64_wide<5>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        case 6: launch_grade_f64_wide<6>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
        default: launch_grade_f64_wide<7>(as, brow, ldn, n, gamma, argmax, st, thr, sel_blk); break;
    }
}

// ---- sustained MFMA rate -----------------------------------------------------
// Every wavefront of a grid of eight wavefronts per CU (two per SIMD, as in
// the grade kernels) runs CH independent accumulation chains of one MFMA
// form on register operands, no memory traffic in the loop: the rate it
// reaches is the ceiling of a kernel built on that form on this part, the
// figure the grade kernels' measured rates compare with beside the nominal
// peak.  The operands are perturbed per iteration (no loop-invariant
// products) and every accumulator is written out at the end.
constexpr int MC_CH = 4;
__global__ __launch_bounds__(256) void mfma_rate_f64(int iters, double *sink) {
    const int lane = threadIdx.x & 63;
    double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
    doublex4 acc[MC_CH];
#pragma unroll
    for (int c = 0; c < MC_CH; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; it += 16) {   // 16 x MC_CH products per trip: the loop overhead is noise
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int c = 0; c < MC_CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        a = a * 0.999999 + 1e-9;
    }
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < MC_CH; ++c) t += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}
__global__ __launch_bounds__(256) void mfma_rate_i8(int iters, double *sink) {
    const int lane = threadIdx.x & 63;
    i32x4 a = {lane, 3 * lane, 5 * lane, 7 * lane}, b = {1, 2, 3, 4};
    i32x4 acc[MC_CH];
#pragma unroll
    for (int c = 0; c < MC_CH; ++c) acc[c] = i32x4{0, 0, 0, 0};
    for (int it = 0; it < iters; it += 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int c = 0; c < MC_CH; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[c], 0, 0, 0);
        a[0] ^= it;
    }
    int t = 0;
#pragma unroll
    for (int c = 0; c < MC_CH; ++c) t += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (double)t;
}

double mfma_rate(int kind, int iters, hipStream_t st) {
    MTP_CHECK(kind == 0 || kind == 1, MTP_E_INVAL, "mfma rate: kind 0 (FP64 16x16x4) or 1 (int8 16x16x64)");
    MTP_CHECK(iters > 0 && iters <= (1 << 24), MTP_E_INVAL, "mfma rate: iters in 1 .. 2^24");
    iters = (iters + 15) / 16 * 16;   // whole trips of the unrolled loop
    int dev = 0, cus = 0;
    MTP_HIP(hipGetDevice(&dev));
    MTP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned blocks = (unsigned)cus * 2;   // 2 x 256 threads = eight wavefronts per CU
    DevBuf sink;
    sink.ensure(sizeof(double) * blocks * 256);
    hipEvent_t e0, e1;
    MTP_HIP(hipEventCreate(&e0));
    MTP_HIP(hipEventCreate(&e1));
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {   // the first launch warms the clocks up
        MTP_HIP(hipEventRecord(e0, st));
        if (kind == 0)
            hipLaunchKernelGGL(mfma_rate_f64, dim3(blocks), dim3(256), 0, st, iters, sink.as<double>());
        else
            hipLaunchKernelGGL(mfma_rate_i8, dim3(blocks), dim3(256), 0, st, iters, sink.as<double>());
        MTP_HIP(hipEventRecord(e1, st));
        MTP_HIP(hipEventSynchronize(e1));
        MTP_HIP(hipEventElapsedTime(&ms, e0, e1));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double per = kind == 0 ? 2.0 * 16 * 16 * 4 : 2.0 * 16 * 16 * 64;   // flops (ops) per MFMA
    const double total = per * MC_CH * (double)iters * blocks * 4;           // 4 wavefronts per block
    return total / (ms * 1e-3) / 1e12;
}

void launch_invert(ActiveSet &as, const double *A, hipStream_t st, DevBuf &work, int *singular_host) {
    const int m = as.m;
    const size_t wsz = (size_t)2 * m * m;
    work.ensure(sizeof(double) * 2 * wsz + 64);
    double *W[2] = {work.as<double>(), work.as<double>() + wsz};
    int32_t *flag = reinterpret_cast<int32_t *>(W[1] + wsz);
    launch_zero(flag, sizeof(int32_t), st);
    const int64_t tot = (int64_t)wsz;
    hipLaunchKernelGGL(gj_setup, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, m, W[0]);
    for (int c = 0; c < m; ++c)
        hipLaunchKernelGGL(gj_step, dim3((unsigned)m), dim3(GJ_T), 0, st, W[c & 1], W[(c + 1) & 1], m, c, flag);
    hipLaunchKernelGGL(gj_extract, dim3((unsigned)(((int64_t)m * m + 255) / 256)), dim3(256), 0, st, W[m & 1], m,
                       as.Ainv.as<double>());
    int32_t h = 0;
    MTP_HIP(hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MTP_HIP(hipStreamSynchronize(st));
    *singular_host = h;
}

void run_maxvol(ActiveSet &as, double *cand, int64_t n_cand, double thr, int max_swaps, int32_t *swap_cand,
                int32_t *swap_col, int32_t *n_swaps, hipStream_t st, DevBuf &work) {
    const int m = as.m;
    const int NB = 256;
    const size_t need = sizeof(double) * ((size_t)n_cand * m + 2 * (size_t)m + (size_t)n_cand + NB) +
                        sizeof(int64_t) * NB + sizeof(MVState) + 256;
    work.ensure(need);
    char *base = static_cast<char *>(work.ptr);
    double *C = reinterpret_cast<double *>(base);
    double *crow = C + (size_t)n_cand * m;
    double *acol = crow + m;
    double *ccol = acol + m;
    double *pv = ccol + n_cand;
    int64_t *pi = reinterpret_cast<int64_t *>(pv + NB);
    MVState *state = reinterpret_cast<MVState *>(pi + NB);
    hipLaunchKernelGGL(mv_init, dim3(1), dim3(64), 0, st, state);
    const int64_t tot = n_cand * m;
    if (tot > 0)
        hipLaunchKernelGGL(gemm_f64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, cand, n_cand,
                           as.Ainv.as<double>(), m, C);
    const int64_t upd = tot > (int64_t)m * m ? tot : (int64_t)m * m;
    const int64_t sv = n_cand > m ? n_cand : m;
    int nb = (int)((tot + AM_T - 1) / AM_T);
    nb = nb < 1 ? 1 : (nb > NB ? NB : nb);
    MVState hs{};
    for (int it = 0; it < max_swaps && tot > 0; ++it) {
        hipLaunchKernelGGL(absmax_partial, dim3(nb), dim3(AM_T), 0, st, C, tot, pv, pi);
        hipLaunchKernelGGL(absmax_final, dim3(1), dim3(64), 0, st, pv, pi, nb, m, thr, max_swaps, C, state, swap_cand,
                           swap_col);
        hipLaunchKernelGGL(mv_save, dim3((unsigned)((sv + 255) / 256)), dim3(256), 0, st, C, n_cand,
                           as.Ainv.as<double>(), m, state, crow, ccol, acol);
        hipLaunchKernelGGL(mv_update, dim3((unsigned)((upd + 255) / 256)), dim3(256), 0, st, C, n_cand,
                           as.Ainv.as<double>(), m, state, crow, ccol, acol);
        hipLaunchKernelGGL(mv_swap, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, as.A.as<double>(), cand, m,
                           state);
        hipLaunchKernelGGL(mv_count, dim3(1), dim3(64), 0, st, state);
        if ((it & 31) == 31) {   // stop enqueueing once converged
            MTP_HIP(hipMemcpyAsync(&hs, state, sizeof(MVState), hipMemcpyDeviceToHost, st));
            MTP_HIP(hipStreamSynchronize(st));
            if (hs.done) break;
        }
    }
    MTP_HIP(hipMemcpyAsync(&hs, state, sizeof(MVState), hipMemcpyDeviceToHost, st));
    MTP_HIP(hipStreamSynchronize(st));
    *n_swaps = hs.swaps;
    prepare_split(as, st);
}

}  // namespace mtp
