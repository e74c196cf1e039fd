// Extrapolation grades and the active set (MLIP-3 paper Sec. II.C-D).
//
//   gamma_i = max_p |(b_i A^-1)_p|, argmax p (lowest index on ties)
//
// FP64 form: v_mfma_f64_16x16x4 tiles.  Mixed form: the FP32 rows b and the
// FP64 A^-1 are split into sums of BF16 terms (x = x_0 + x_1 + x_2, each term
// the BF16 rounding of what is left), and C = sum_{s+t < NS} b_s A_t on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
//
// A block of 512 threads owns 64 rows of C; each wavefront 16 rows and half
// of each pass of 224 columns.  The block keeps a running max / argmax per
// row, so C is never written.  A^-1 (<= m^2 x 8 B) stays L2-resident.
//
// Also here: A^-1 by Gauss-Jordan elimination (FP64, partial pivoting) and
// the MaxVol swap loop with Sherman-Morrison updates (FP64 only).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace mtp {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));   // a 16-byte piece, kept in registers

__device__ inline void better(double v, int c, double &bv, int &bc) {
    if (v > bv || (v == bv && c < bc)) {
        bv = v;
        bc = c;
    }
}

// Result layouts of the two MFMAs (16x16 tile, lane l, register r):
//   f64 16x16x4:       row (l/16) + 4 r, column l % 16
//   f32 16x16x32 bf16: row 4 (l/16) + r, column l % 16

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
__global__ __launch_bounds__(512) void grade_f64(const double *__restrict__ brow, int ldb, int64_t n,
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
            for (int q = 0; q < RA; ++q) {
                const int e = tid + 512 * q;
                const int r = e / GF_KC, k = k0 + e % GF_KC;   // k < ldb: the rows are padded with zeros
                R.a[q] = brow[min(row0 + r, n - 1) * ldb + k];
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
                sA[buf][e / GF_KC][e % GF_KC] = R.a[q];
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

// split of x into NS BF16 terms (round to nearest even at every step)
template <int NS> __device__ inline void split_f32(float x, __bf16 (&t)[NS]) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        t[s] = (__bf16)x;
        x -= (float)t[s];
    }
}

// Ainv split layout: S[term][col][kp] (kp = k padded to KP, col padded to CP),
// so that 8 consecutive k of one column are one 16-byte load.
//
// Block of eight wavefronts, 64 rows; wave w takes rows 16 (w % 4) .. + 16
// and half w / 4 of each pass of 32 HALF columns.  k runs in chunks of 32
// (one MFMA k step) through two LDS buffers: the rows' FP32 chunk is split
// into its BF16 terms as it is stored, the split A^-1 chunk is copied as is.
// Branch-free inner loop as in grade_f64 (clamped loads; the split A^-1 is
// zero past m in k, columns past m are never compared).
constexpr int GB_KC = 32, GB_KPAD = GB_KC + 8;   // +8 bf16: 80-byte rows spread the LDS banks
template <int NS, int HALF>
__global__ __launch_bounds__(512) void grade_bf16(const float *__restrict__ brow, int ldb, int64_t n,
                                                  const __bf16 *__restrict__ S, int m, int KP, int CP, double *gamma,
                                                  int32_t *argmax, double thr, int32_t *sel_blk) {
    constexpr int CT = 32 * HALF;
    __shared__ __attribute__((aligned(16))) __bf16 sA[2][NS][GF_ROWS][GB_KPAD];
    __shared__ __attribute__((aligned(16))) __bf16 sB[2][NS][CT][GB_KPAD];
    __shared__ double s_best[2][GF_ROWS];
    __shared__ int s_idx[2][GF_ROWS];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rg = wave & 3, half = wave >> 2;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * GF_ROWS;
    const int64_t term = (int64_t)CP * KP;
    const int nchunk = KP / GB_KC;
    // global -> register staging: A, one float4 per thread (row tid / 8, k 4 (tid % 8));
    // B, 16-byte pieces e = tid + 512 q of (term, column, k group of 8)
    constexpr int NBP = NS * CT * (GB_KC / 8);
    constexpr int RB = (NBP + 511) / 512;
    double best[4] = {-1.0, -1.0, -1.0, -1.0};
    int bidx[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    for (int ct0 = 0; ct0 < m; ct0 += CT) {
        const int cb0 = half * HALF;
        floatx4 acc[HALF];
#pragma unroll
        for (int c = 0; c < HALF; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
        float4 ra;
        u32x4 rb[RB];
        auto fetch = [&](int ch) {
            const int k0 = ch * GB_KC;
            const int r = tid >> 3, k = k0 + 4 * (tid & 7);
            ra = *reinterpret_cast<const float4 *>(brow + min(row0 + r, n - 1) * ldb + k);
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int e = tid + 512 * q;
                const int t = e / (CT * 4), rem = e % (CT * 4), c = rem >> 2, kg = rem & 3;
                const int col = min(ct0 + c, CP - 1);
                if (q < RB - 1 || e < NBP)
                    rb[q] = *reinterpret_cast<const u32x4 *>(S + t * term + (int64_t)col * KP + k0 + 8 * kg);
            }
        };
        auto store = [&](int buf) {
            const int r = tid >> 3, k = 4 * (tid & 7);
            const float v[4] = {ra.x, ra.y, ra.z, ra.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                __bf16 t[NS];
                split_f32<NS>(v[e], t);
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2) sA[buf][s2][r][k + e] = t[s2];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int e = tid + 512 * q;
                if (q < RB - 1 || e < NBP) {
                    const int t = e / (CT * 4), rem = e % (CT * 4), c = rem >> 2, kg = rem & 3;
                    *reinterpret_cast<u32x4 *>(&sB[buf][t][c][8 * kg]) = rb[q];
                }
            }
        };
        __syncthreads();
        fetch(0);
        store(0);
        __syncthreads();
        for (int ch = 0; ch < nchunk; ++ch) {
            const int buf = ch & 1;
            if (ch + 1 < nchunk) fetch(ch + 1);
            bf16x8 A[NS];
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) A[s2] = *reinterpret_cast<const bf16x8 *>(&sA[buf][s2][rg * 16 + lr][8 * lk]);
#pragma unroll
            for (int c = 0; c < HALF; ++c) {
#pragma unroll
                for (int t = 0; t < NS; ++t) {
                    const bf16x8 B = *reinterpret_cast<const bf16x8 *>(&sB[buf][t][(cb0 + c) * 16 + lr][8 * lk]);
#pragma unroll
                    for (int s2 = 0; s2 + t < NS; ++s2)
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s2], B, acc[c], 0, 0, 0);
                }
            }
            if (ch + 1 < nchunk) store(buf ^ 1);
            __syncthreads();
        }
#pragma unroll
        for (int c = 0; c < HALF; ++c) {
            const int col = ct0 + (cb0 + c) * 16 + lr;
            if (col < m)
#pragma unroll
                for (int r = 0; r < 4; ++r) better((double)fabsf(acc[c][r]), col, best[r], bidx[r]);
        }
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double ov = __shfl_xor(best[r], o, 64);
            const int oc = __shfl_xor(bidx[r], o, 64);
            better(ov, oc, best[r], bidx[r]);
        }
    if (lr == 0)   // bf16 layout: row 4 (lane / 16) + r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s_best[half][rg * 16 + 4 * lk + r] = best[r];
            s_idx[half][rg * 16 + 4 * lk + r] = bidx[r];
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

__global__ void split_ainv(const double *Ainv, int m, int KP, int CP, int NS, __bf16 *S) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)CP * KP) return;
    const int col = (int)(idx / KP), k = (int)(idx % KP);
    double x = (col < m && k < m) ? Ainv[(int64_t)k * m + col] : 0.0;
    const int64_t term = (int64_t)CP * KP;
    for (int s = 0; s < NS; ++s) {
        const __bf16 t = (__bf16)(float)x;
        S[s * term + idx] = t;
        x -= (double)(float)t;
    }
}

// ---- Gauss-Jordan inverse (one block) ----------------------------------------
constexpr int GJ_T = 1024;
__global__ __launch_bounds__(GJ_T) void gauss_jordan(double *W, int m, int32_t *singular) {
    // W is m x 2m: [A | I] -> [I | A^-1]
    __shared__ double sv[GJ_T];
    __shared__ int si[GJ_T];
    __shared__ int piv;
    const int n2 = 2 * m;
    for (int c = 0; c < m; ++c) {
        double bv = -1.0;
        int bi = m;
        for (int r = c + threadIdx.x; r < m; r += GJ_T) {
            const double v = fabs(W[(int64_t)r * n2 + c]);
            if (v > bv) {
                bv = v;
                bi = r;
            }
        }
        sv[threadIdx.x] = bv;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int w = GJ_T / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                const double ov = sv[threadIdx.x + w];
                const int oi = si[threadIdx.x + w];
                if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                    sv[threadIdx.x] = ov;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            piv = si[0];
            if (!(sv[0] > 1e-300)) *singular = 1;
        }
        __syncthreads();
        if (*singular) return;   // uniform: every thread sees the same flag
        const int p = piv;
        if (p != c)
            for (int k = threadIdx.x; k < n2; k += GJ_T) {
                const double t = W[(int64_t)p * n2 + k];
                W[(int64_t)p * n2 + k] = W[(int64_t)c * n2 + k];
                W[(int64_t)c * n2 + k] = t;
            }
        __syncthreads();
        const double inv = 1.0 / W[(int64_t)c * n2 + c];
        __syncthreads();
        for (int k = threadIdx.x; k < n2; k += GJ_T) W[(int64_t)c * n2 + k] *= inv;
        __syncthreads();
        for (int64_t e = threadIdx.x; e < (int64_t)m * n2; e += GJ_T) {
            const int r = (int)(e / n2), k = (int)(e % n2);
            if (r == c || k == c) continue;
            const double f = W[(int64_t)r * n2 + c];
            if (f != 0.0) W[e] -= f * W[(int64_t)c * n2 + k];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < m; r += GJ_T)
            if (r != c) W[(int64_t)r * n2 + c] = 0.0;
        __syncthreads();
    }
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

int split_terms() { return 3; }

void prepare_split(ActiveSet &as, hipStream_t st) {
    const int m = as.m;
    const int KP = (m + 31) / 32 * 32, CP = (m + 15) / 16 * 16;
    const int NS = split_terms();
    as.Ainv32.ensure(sizeof(__bf16) * (size_t)NS * CP * KP);
    const int64_t tot = (int64_t)CP * KP;
    hipLaunchKernelGGL(split_ainv, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, as.Ainv.as<double>(), m, KP,
                       CP, NS, as.Ainv32.as<__bf16>());
}

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
static void launch_grade_h(const ActiveSet &as, int precision, const void *brow, int ldb, int64_t n, double *gamma,
                           int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk) {
    const dim3 grid((unsigned)((n + GF_ROWS - 1) / GF_ROWS));
    if (precision == MTP_FP64) {
        hipLaunchKernelGGL(grade_f64<HALF>, grid, dim3(512), 0, st, static_cast<const double *>(brow), ldb, n,
                           as.Ainv.as<double>(), as.m, gamma, argmax, thr, sel_blk);
    } else {
        const int KP = (as.m + 31) / 32 * 32, CP = (as.m + 15) / 16 * 16;
        hipLaunchKernelGGL((grade_bf16<3, HALF>), grid, dim3(512), 0, st, static_cast<const float *>(brow), ldb, n,
                           as.Ainv32.as<__bf16>(), as.m, KP, CP, gamma, argmax, thr, sel_blk);
    }
}

void launch_grade(const ActiveSet &as, int precision, const void *brow, int ldb, int64_t n, double *gamma,
                  int32_t *argmax, hipStream_t st, double thr, int32_t *sel_blk) {
    static_assert(GRADE_ROWS == GF_ROWS, "preselection blocks are grade blocks");
    if (n == 0) return;
    MTP_CHECK(ldb >= (as.m + 31) / 32 * 32, MTP_E_INVAL, "grade: row stride below the padded row length");
    switch (grade_half(as.m)) {
        case 1: launch_grade_h<1>(as, precision, brow, ldb, n, gamma, argmax, st, thr, sel_blk); break;
        case 2: launch_grade_h<2>(as, precision, brow, ldb, n, gamma, argmax, st, thr, sel_blk); break;
        case 3: launch_grade_h<3>(as, precision, brow, ldb, n, gamma, argmax, st, thr, sel_blk); break;
        case 4: launch_grade_h<4>(as, precision, brow, ldb, n, gamma, argmax, st, thr, sel_blk); break;
        case 5: launch_grade_h<5>(as, precision, brow, ldb, n, gamma, argmax, st, thr, sel_blk); break;
        case 6: launch_grade_h<6>(as, precision, brow, ldb, n, gamma, argmax, st, thr, sel_blk); break;
        default: launch_grade_h<7>(as, precision, brow, ldb, n, gamma, argmax, st, thr, sel_blk); break;
    }
}

void launch_invert(ActiveSet &as, const double *A, hipStream_t st, DevBuf &work, int *singular_host) {
    const int m = as.m;
    work.ensure(sizeof(double) * (size_t)2 * m * m + 64);
    double *W = work.as<double>();
    int32_t *flag = reinterpret_cast<int32_t *>(W + (size_t)2 * m * m);
    launch_zero(flag, sizeof(int32_t), st);
    const int64_t tot = (int64_t)2 * m * m;
    hipLaunchKernelGGL(gj_setup, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, m, W);
    hipLaunchKernelGGL(gauss_jordan, dim3(1), dim3(GJ_T), 0, st, W, m, flag);
    hipLaunchKernelGGL(gj_extract, dim3((unsigned)(((int64_t)m * m + 255) / 256)), dim3(256), 0, st, W, m,
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
