// Fused per-neighborhood kernel: radial functions -> moments -> contraction
// -> site energy -> dV/dM -> pair gradients, virial and (optionally) the row
// b_i = dV_i/dtheta.  Included by one generated translation unit per level.
//
// Work decomposition: LANES consecutive lanes of a wavefront share one
// neighborhood.  Each lane walks every LANES-th pair of the list and keeps
// its own partial moments in registers; a butterfly of cross-lane shuffles
// then gives every lane the full moments.  The contraction program (Level<L>,
// generated at build time) runs in registers.  The pair loop is walked a
// second time for the gradients, one neighbor species after the other, so
// the radial-coefficient part of b_i needs only N_rad x N_polyn accumulators.
//
// Pair gradient (paper eqs. 3-4; V from eq. 2):
//   g_ij = dV_i/dr_ij = sum_mu [ f'_mu(r) P_mu r_hat + f_mu(r) grad P_mu ],
//   P_mu(r) = sum_{k in mu} (dV/dM_k) x^a y^b z^c  (k = component (mu; a,b,c)).
// b-row entries of c (eq. 4): dV_i/dc^(beta)_{mu,z_i,z} = sum_{j: z_j = z} Q_beta(r_ij) P_mu(r_ij),
// Q_beta = T_beta(x) (R_cut - r)^2.
//
// Rows are FP64 in every form and stored column-major: entry (i, k) at
// brow[k * ldn + i], so that the lanes of a wavefront (consecutive
// neighborhoods) write consecutive words of one column.
#pragma once

#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernel_args.hpp"

namespace mtp {

template <int L> struct Level;

namespace efs {

template <typename T> __device__ inline T xor_shuffle(T v, int mask) { return __shfl_xor(v, mask, 64); }

// Reduce-scatter over the K lanes of a group (sub = lane % K): afterwards
// v[0 .. M/K) of lane sub holds the group totals of v[sub M/K .. (sub+1) M/K).
// Each round halves the live values (the lane whose bit O is set keeps the
// upper half), so it takes M (1 - 1/K) shuffles instead of the M log2 K of a
// butterfly all-reduce.
template <typename T, int M, int N, int O> __device__ inline void rs_step(T (&v)[M], int sub) {
    if constexpr (O >= 1) {
        const bool up = (sub & O) != 0;
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
            const T send = up ? v[i] : v[i + N / 2];
            const T keep = up ? v[i + N / 2] : v[i];
            v[i] = keep + xor_shuffle(send, O);
        }
        rs_step<T, M, N / 2, O / 2>(v, sub);
    }
}
template <typename T, int M, int K> __device__ inline void reduce_scatter(T (&v)[M], int sub) {
    static_assert(M % K == 0, "reduce_scatter: M must be a multiple of K");
    rs_step<T, M, M, K / 2>(v, sub);
}

// monomials x^a y^b z^c, a+b+c <= 3, in the order of monomial_index()
template <typename T> __device__ inline void monomials(T x, T y, T z, T (&m)[20]) {
    m[0] = T(1); m[1] = x; m[2] = y; m[3] = z;
    m[4] = x * x; m[5] = x * y; m[6] = x * z; m[7] = y * y; m[8] = y * z; m[9] = z * z;
    m[10] = m[4] * x; m[11] = m[4] * y; m[12] = m[4] * z; m[13] = m[7] * x; m[14] = m[5] * z;
    m[15] = m[9] * x; m[16] = m[7] * y; m[17] = m[7] * z; m[18] = m[9] * y; m[19] = m[9] * z;
}

}  // namespace efs

// theta = [xi_0 (n_types) | xi_alpha (n_lin) | c] in the arithmetic type T
template <typename T> __device__ inline const T *theta_of(const EfsArgs &a);
template <> __device__ inline const double *theta_of<double>(const EfsArgs &a) { return a.th64; }
template <> __device__ inline const float *theta_of<float>(const EfsArgs &a) { return a.th32; }
template <typename T> __device__ inline const T *xi0_of(const EfsArgs &a) { return theta_of<T>(a); }
template <typename T> __device__ inline const T *xi_of(const EfsArgs &a) { return theta_of<T>(a) + a.n_types; }
template <typename T> __device__ inline const T *coef_of(const EfsArgs &a) {
    return theta_of<T>(a) + a.n_types + a.n_lin;
}

template <typename T> struct XiPtr {      // xi_alpha, read where the program needs it
    const T *p;
    __device__ T operator[](int k) const { return p[k]; }
};

// Per-neighborhood context shared by the pair kernels.
struct AtomCtx {
    bool live;
    int64_t slot, atom;
    int zi, ntot;
    int tc[MAX_TYPES];
    const double *rp;
};

// BS: the launch's block size, a compile-time constant (blockDim.x is read
// from the dispatch packet: one more dependent load before the first real one)
template <int K, int BS = 256> __device__ inline AtomCtx atom_ctx(const EfsArgs &a, int64_t blk = -1) {
    AtomCtx c;
    const int nt = a.n_types;
    c.slot = (blk < 0 ? (int64_t)blockIdx.x : blk) * (BS / K) + threadIdx.x / K;
    c.live = c.slot < a.n_atoms;
    c.atom = c.live ? (a.atom_list ? (int64_t)a.atom_list[c.slot] : c.slot) : 0;
    int zi = c.live ? a.type[c.atom] : 0;
    c.zi = zi < 0 ? 0 : (zi >= nt ? nt - 1 : zi);
    c.ntot = 0;
#pragma unroll
    for (int t = 0; t < MAX_TYPES; ++t) {
        c.tc[t] = (c.live && t < nt) ? a.tcnt[c.atom * nt + t] : 0;
        c.ntot += c.tc[t];
    }
    c.rp = a.r + c.atom * (int64_t)a.max_nbrs * 3;
    return c;
}

// neighbors of species t, re-read from the (cached) counts: a runtime index
// into c.tc would put the whole context in scratch memory
template <typename A> __device__ inline int tcount(const A &a, const AtomCtx &c, int t) {
    return c.live ? a.tcnt[c.atom * a.n_types + t] : 0;
}

// The radial coefficients c_{mu, z_i, z_j, beta} in LDS as
// [mu][beta][z_i][z_j], the species padded to MAX_TYPES: the lanes of a
// wavefront, whose pairs have different (z_i, z_j), read one (mu, beta) at a
// time from one 16-word row (no bank conflicts; the parameter order
// [mu][z_i][z_j][beta] puts them NPOLY words apart), and beta steps by a
// constant offset.
constexpr int COEF_TT = MAX_TYPES * MAX_TYPES;
template <typename T, int NR, int BS = 256> __device__ inline void load_coefs(const EfsArgs &a, T *c_s) {
    const T *cg = coef_of<T>(a);
    const int nt = a.n_types, ntt = nt * nt;
    const int ncoef = NR * ntt * NPOLY;
    for (int k = threadIdx.x; k < ncoef; k += BS) {
        const int b = k % NPOLY, pair = (k / NPOLY) % ntt, mu = k / (NPOLY * ntt);
        c_s[(mu * NPOLY + b) * COEF_TT + (pair / nt) * MAX_TYPES + pair % nt] = cg[k];
    }
    __syncthreads();
}
template <typename T> struct CoefRow {   // c_{mu, z_i, z_j, beta} over beta, from the LDS copy
    const T *p;
    __device__ T operator[](int b) const { return p[b * COEF_TT]; }
};
template <typename T> __device__ inline CoefRow<T> coef_row(const T *c_s, int mu, int zi, int zj, int) {
    return CoefRow<T>{c_s + mu * NPOLY * COEF_TT + zi * MAX_TYPES + zj};
}

// ---- kernel 1: moments (eq. 3), LANES lanes per neighborhood -------------
// Moments of the neighborhood of c, reduce-scattered over its K lanes: on
// return M[i] of lane sub holds component sub NCP/K + i (NCP = NC padded to
// a multiple of K).  c_s: the radial coefficients, already in LDS.
template <typename T, int L, int K>
__device__ inline void moments_scattered(const EfsArgs &a, const AtomCtx &c, const T *c_s,
                                         T (&M)[(Level<L>::NC + K - 1) / K * K]) {
    using LV = Level<L>;
    constexpr int NC = LV::NC, NR = LV::NRAD;
    const int nt = a.n_types;
    const int sub = threadIdx.x % K;
    const T rc = T(a.r_cut);
    const T xs = T(2.0 / (a.r_cut - a.r_min));
    const T x0 = T(-(a.r_min + a.r_cut) / (a.r_cut - a.r_min));
    constexpr int NCP = (NC + K - 1) / K * K;   // padded for the reduce-scatter
#pragma unroll
    for (int k = 0; k < NCP; ++k) M[k] = T(0);
    int zj = 0, tend = c.tc[0];
    // the next pair vector is loaded while the current one is used
    double nx = 0.0, ny = 0.0, nz = 0.0;
    if (sub < c.ntot) {
        nx = c.rp[3 * sub];
        ny = c.rp[3 * sub + 1];
        nz = c.rp[3 * sub + 2];
    }
    for (int p = sub; p < c.ntot; p += K) {
        while (p >= tend && zj < nt - 1) tend += tcount(a, c, ++zj);
        const T x = T(nx), y = T(ny), z = T(nz);
        if (p + K < c.ntot) {
            nx = c.rp[3 * (p + K)];
            ny = c.rp[3 * (p + K) + 1];
            nz = c.rp[3 * (p + K) + 2];
        }
        const T r = sqrt(x * x + y * y + z * z);
        if (!(r < rc)) continue;
        T fm[NR];
        {
            const T u = fma(r, xs, x0), d = rc - r, cut = d * d;
            T Tb[NPOLY];
            Tb[0] = T(1);
            Tb[1] = u;
#pragma unroll
            for (int b = 2; b < NPOLY; ++b) Tb[b] = fma(T(2) * u, Tb[b - 1], -Tb[b - 2]);
#pragma unroll
            for (int mu = 0; mu < NR; ++mu) {
                const CoefRow<T> cm = coef_row(c_s, mu, c.zi, zj, nt);
                T s = T(0);
#pragma unroll
                for (int b = 0; b < NPOLY; ++b) s = fma(cm[b], Tb[b], s);
                fm[mu] = s * cut;
            }
        }
        T mono[20];
        efs::monomials(x, y, z, mono);
#pragma unroll
        for (int k = 0; k < NC; ++k) M[k] = fma(fm[LV::comp_mu[k]], mono[LV::comp_mono[k]], M[k]);
    }
    efs::reduce_scatter<T, NCP, K>(M, sub);
}

template <typename T, int L, int K>
__global__ __launch_bounds__(256) void efs_moments(const EfsArgs a) {
    using LV = Level<L>;
    constexpr int NC = LV::NC, NR = LV::NRAD;
    constexpr int NCP = (NC + K - 1) / K * K;
    __shared__ T c_s[NR * MAX_TYPES * MAX_TYPES * NPOLY];
    load_coefs<T, NR>(a, c_s);
    const int sub = threadIdx.x % K;
    const AtomCtx c = atom_ctx<K>(a);
    T M[NCP];
    moments_scattered<T, L, K>(a, c, c_s, M);
    if (c.live) {
        T *out = static_cast<T *>(a.mbuf);
#pragma unroll
        for (int i = 0; i < NCP / K; ++i) {
            const int k = sub * (NCP / K) + i;
            if (k < NC) out[(int64_t)k * a.n_atoms + c.slot] = M[i];
        }
    }
}

// ---- kernel 2: contraction, site energy (eq. 2), dV/dM -------------------
// One block holds 64 neighborhoods (one per lane) and four (or eight)
// wavefronts; the graphs of the contraction program are split into four and
// into eight parts at build time (Level<L>::graph_part, graph_part8).
// Wavefront w evaluates the graph values of part w, all exchange them through
// LDS, each runs the (short) trie walk for V, B_alpha and dV/dg, and
// wavefront w runs the reverse pass of part w.  The partial dV/dM are added
// in LDS in a fixed order.
template <typename T> struct ColLoad {   // component k of one neighborhood, [k][n] layout
    const T *p;
    int64_t s;
    __device__ T operator[](int k) const { return p[k * s]; }
};
template <typename T> struct LdsSink {   // receives B_alpha into [alpha][64] in LDS
    T *p;
    __device__ T &operator[](int k) const { return p[k * 64]; }
};
// receives B_alpha straight into column c0 + alpha of the FP64 rows (when
// staging them would not fit in LDS): a uniform column base plus the lane's
// row index, consecutive lanes writing consecutive words
struct ColSink {
    double *p;
    int64_t s;
    int c0;
    uint32_t row;
    bool on;
    struct Ref {
        double *col;
        uint32_t row;
        bool on;
        __device__ void operator=(const double &v) const {
            if (on) col[row] = v;
        }
    };
    __device__ Ref operator[](int k) const { return Ref{p + (int64_t)(c0 + k) * s, row, on}; }
};
struct NoSink {
    struct Ref {
        template <typename V> __device__ void operator=(const V &) const {}
    };
    __device__ Ref operator[](int) const { return Ref{}; }
};

template <typename T> struct LdsCol {   // component k of one neighborhood, [k][64] in LDS
    const T *p;
    __device__ T operator[](int k) const { return p[k * 64]; }
};

// Rows of graph values / B_alpha staged in LDS: the graph values, and with
// rows wanted (WB) B_alpha in the same place once the graph values are read,
// when that fits in STAGE_BYTES (else B_alpha goes straight to memory).
constexpr int STAGE_BYTES = 64 * 1024;
template <typename T, int L, bool WB> constexpr bool stage_b() {
    return WB && Level<L>::NLIN * 64 * (int)sizeof(T) <= STAGE_BYTES;
}
template <typename T, int L, bool WB> constexpr int sg_rows() {
    return stage_b<T, L, WB>() && Level<L>::NLIN > Level<L>::NGRAPH ? Level<L>::NLIN : Level<L>::NGRAPH;
}

// The contraction of the 64 neighborhoods of block blk (a block of NW = 4
// or 8 wavefronts), the moments read through M; sg, sdm: LDS scratch.
// ALIAS: sdm shares its storage with the moments M (they are dead once every
// wavefront has finished its reverse part, which a barrier makes sure of).
// WB: B_alpha goes into the rows (FP64 only: rows are always FP64), staged
// in sg and written column by column (64 consecutive rows per store).
template <typename T, int L, bool WB, typename MA, int NW = 4, bool ALIAS = false>
__device__ inline void contract_body(const EfsArgs &a, int64_t blk, const MA &M,
                                     T (&sg)[sg_rows<T, L, WB>()][64], T (&sdm)[Level<L>::NC][64]) {
    using LV = Level<L>;
    constexpr int NC = LV::NC, NG = LV::NGRAPH;
    static_assert(LV::NPART == 4 && LV::NPART8 == 8 && (NW == 4 || NW == 8), "four or eight parts");
    static_assert(!WB || sizeof(T) == sizeof(double), "rows are FP64");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t slot = blk * 64 + lane;
    const bool live = slot < a.n_atoms;
    const int64_t sl = live ? slot : 0;
    if constexpr (WB) {
        // the rows' constant entries, in whole columns of 64 rows: the species
        // one-hot, then zeros from column nt + NL on (the c part's blocks and
        // the padding; the pair pass writes the neighborhood's own c block
        // over them afterwards).  Issued first, so that they drain while the
        // graph values are computed (no vector memory load follows that
        // would wait for them)
        if (live) {
            const int ntp = a.n_types;
            const int64_t atom = a.atom_list ? (int64_t)a.atom_list[slot] : slot;
            int zi = a.type[atom];
            zi = zi < 0 ? 0 : (zi >= ntp ? ntp - 1 : zi);
            double *rowp = a.brow + sl;
            const int c0 = ntp + LV::NLIN;
            for (int k = wave; k < ntp + a.ldb - c0; k += NW) {
                const int col = k < ntp ? k : c0 + (k - ntp);
                rowp[(int64_t)col * a.ldn] = k == zi ? 1.0 : 0.0;
            }
        }
    }
    {
        T g[NG];
        if constexpr (NW == 4) {
            switch (wave) {
                case 0: LV::template graphs_part<0>(M, g); break;
                case 1: LV::template graphs_part<1>(M, g); break;
                case 2: LV::template graphs_part<2>(M, g); break;
                default: LV::template graphs_part<3>(M, g); break;
            }
        } else {
            switch (wave) {
                case 0: LV::template graphs_part8<0>(M, g); break;
                case 1: LV::template graphs_part8<1>(M, g); break;
                case 2: LV::template graphs_part8<2>(M, g); break;
                case 3: LV::template graphs_part8<3>(M, g); break;
                case 4: LV::template graphs_part8<4>(M, g); break;
                case 5: LV::template graphs_part8<5>(M, g); break;
                case 6: LV::template graphs_part8<6>(M, g); break;
                default: LV::template graphs_part8<7>(M, g); break;
            }
        }
#pragma unroll
        for (int G = 0; G < NG; ++G)
            if ((NW == 4 ? LV::graph_part[G] : LV::graph_part8[G]) == wave) sg[G][lane] = g[G];
    }
    __syncthreads();
    T gin[NG], dg[NG];
#pragma unroll
    for (int G = 0; G < NG; ++G) gin[G] = sg[G][lane];
    T V = T(0);
    const int nt = a.n_types;
    const XiPtr<T> xi{xi_of<T>(a)};
    if constexpr (stage_b<T, L, WB>()) {
        __syncthreads();   // every wavefront has read the graph values: sg takes B_alpha
        if (wave == 0) {
            LV::template trie<T, true>(gin, xi, LdsSink<T>{&sg[0][lane]}, dg, V);
        } else {
            LV::template trie<T, false>(gin, xi, NoSink{}, dg, V);
        }
    } else if constexpr (WB) {
        if (wave == 0) {
            LV::template trie<T, true>(gin, xi, ColSink{a.brow, a.ldn, nt, (uint32_t)sl, live}, dg, V);
        } else {
            LV::template trie<T, false>(gin, xi, NoSink{}, dg, V);
        }
    } else {
        LV::template trie<T, false>(gin, xi, NoSink{}, dg, V);
    }
    T dMp[NC];
    if constexpr (NW == 4) {
        switch (wave) {
            case 0: LV::template reverse_part<0>(M, dg, dMp); break;
            case 1: LV::template reverse_part<1>(M, dg, dMp); break;
            case 2: LV::template reverse_part<2>(M, dg, dMp); break;
            default: LV::template reverse_part<3>(M, dg, dMp); break;
        }
    } else {
        switch (wave) {
            case 0: LV::template reverse_part8<0>(M, dg, dMp); break;
            case 1: LV::template reverse_part8<1>(M, dg, dMp); break;
            case 2: LV::template reverse_part8<2>(M, dg, dMp); break;
            case 3: LV::template reverse_part8<3>(M, dg, dMp); break;
            case 4: LV::template reverse_part8<4>(M, dg, dMp); break;
            case 5: LV::template reverse_part8<5>(M, dg, dMp); break;
            case 6: LV::template reverse_part8<6>(M, dg, dMp); break;
            default: LV::template reverse_part8<7>(M, dg, dMp); break;
        }
    }
    if constexpr (ALIAS) __syncthreads();   // every reverse part has read M
    for (int w = 0; w < NW; ++w) {
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < NC; ++k) sdm[k][lane] = w == 0 ? dMp[k] : sdm[k][lane] + dMp[k];
        }
        __syncthreads();
    }
    if constexpr (stage_b<T, L, WB>()) {   // B_alpha (written to sg by wavefront 0 before the barriers above)
        double *col = a.brow + (int64_t)nt * a.ldn + sl;
        if (live)
            for (int k = wave; k < LV::NLIN; k += NW) col[(int64_t)k * a.ldn] = sg[k][lane];
    }
    if (live) {
        T *dout = static_cast<T *>(a.dmbuf);
        for (int k = wave; k < NC; k += NW) dout[(int64_t)k * a.n_atoms + slot] = sdm[k][lane];
        if (wave == 0 && a.site_e) {
            const int64_t atom = a.atom_list ? (int64_t)a.atom_list[slot] : slot;
            int zi = a.type[atom];
            zi = zi < 0 ? 0 : (zi >= nt ? nt - 1 : zi);
            a.site_e[atom] = double(V) + double(xi0_of<T>(a)[zi]);
        }
    }
}

template <typename T, int L, bool WB>
__global__ __launch_bounds__(256) void efs_contract(const EfsArgs a) {
    using LV = Level<L>;
    __shared__ T sg[sg_rows<T, L, WB>()][64];
    __shared__ T sdm[LV::NC][64];
    const int64_t slot = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const int64_t sl = slot < a.n_atoms ? slot : 0;
    contract_body<T, L, WB>(a, blockIdx.x, ColLoad<T>{static_cast<const T *>(a.mbuf) + sl, a.n_atoms}, sg, sdm);
}

// Kernels 1 and 2 in one launch (four lanes per neighborhood: the 256
// threads of a block hold the same 64 neighborhoods in both phases): the
// reduce-scattered moments go to LDS instead of memory, and after one
// barrier the contraction reads them there.  dV/dM reuses the moments'
// LDS and B_alpha the graph values', so a block holds the radial
// coefficients, the moments and max(graph values, B_alpha) only (78 KB at
// level 16 in FP64 with rows, 45 KB without: two blocks per CU).
template <typename T, int L, bool WB>
__global__ __launch_bounds__(256) void efs_moments_contract(const EfsArgs a) {
    using LV = Level<L>;
    constexpr int K = 4, NC = LV::NC, NR = LV::NRAD;
    constexpr int NCP = (NC + K - 1) / K * K;
    __shared__ T c_s[NR * MAX_TYPES * MAX_TYPES * NPOLY];
    __shared__ T sM[NCP][64];
    __shared__ T sg[sg_rows<T, L, WB>()][64];
    load_coefs<T, NR>(a, c_s);
    const int sub = threadIdx.x % K;
    const AtomCtx c = atom_ctx<K>(a);
    {
        T M[NCP];
        moments_scattered<T, L, K>(a, c, c_s, M);
        const int la = threadIdx.x / K;
#pragma unroll
        for (int i = 0; i < NCP / K; ++i) sM[sub * (NCP / K) + i][la] = M[i];
    }
    __syncthreads();
    contract_body<T, L, WB, LdsCol<T>, 4, true>(a, blockIdx.x, LdsCol<T>{&sM[0][threadIdx.x & 63]}, sg,
                                                 reinterpret_cast<T (&)[NC][64]>(sM));
}

// The same with eight wavefronts (512 threads, eight lanes per neighborhood
// for the moments) and the eight-part contraction program: 64 neighborhoods
// per block as before, but two wavefronts per SIMD instead of one while the
// straight-line contraction runs.
template <typename T, int L, bool WB>
__global__ __launch_bounds__(512) void efs_moments_contract8(const EfsArgs a) {
    using LV = Level<L>;
    constexpr int K = 8, NC = LV::NC, NR = LV::NRAD;
    constexpr int NCP = (NC + K - 1) / K * K;
    __shared__ T c_s[NR * MAX_TYPES * MAX_TYPES * NPOLY];
    __shared__ T sM[NCP][64];
    __shared__ T sg[sg_rows<T, L, WB>()][64];
    load_coefs<T, NR, 512>(a, c_s);
    const int sub = threadIdx.x % K;
    const AtomCtx c = atom_ctx<K, 512>(a);
    {
        T M[NCP];
        moments_scattered<T, L, K>(a, c, c_s, M);
        const int la = threadIdx.x / K;
#pragma unroll
        for (int i = 0; i < NCP / K; ++i) sM[sub * (NCP / K) + i][la] = M[i];
    }
    __syncthreads();
    contract_body<T, L, WB, LdsCol<T>, 8, true>(a, blockIdx.x, LdsCol<T>{&sM[0][threadIdx.x & 63]}, sg,
                                                 reinterpret_cast<T (&)[NC][64]>(sM));
}

// Chebyshev values (and derivatives) at u for the radial basis (eq. 4)
template <typename T, bool DERIV>
__device__ inline void chebyshev(T u, T (&Tb)[NPOLY], T (&dT)[NPOLY]) {
    Tb[0] = T(1);
    Tb[1] = u;
    if (DERIV) {
        dT[0] = T(0);
        dT[1] = T(1);
    }
#pragma unroll
    for (int b = 2; b < NPOLY; ++b) {
        Tb[b] = fma(T(2) * u, Tb[b - 1], -Tb[b - 2]);
        if (DERIV) dT[b] = fma(T(2) * u, dT[b - 1], fma(T(2), Tb[b - 1], -dT[b - 2]));
    }
}

// dE/dM of the block's neighborhoods in LDS, [k][neighborhood in block]: the
// K lanes of a neighborhood read the same word (broadcast); in registers
// they would cost 2 NC VGPRs per lane.  TD: the type dV/dM was computed in
// (FP64 when the FP32 pair gradients of the mixed form follow an FP64
// contraction that also fed the rows).
template <typename T, int NC, int K, typename TD = T>
__device__ inline void load_dm(const EfsArgs &a, const AtomCtx &c, int sub, T (&s_dm)[NC][256 / K]) {
    const TD *din = static_cast<const TD *>(a.dmbuf);
    const int la = threadIdx.x / K;
    for (int k = sub; k < NC; k += K) s_dm[k][la] = c.live ? T(din[(int64_t)k * a.n_atoms + c.slot]) : T(0);
    __syncthreads();
}

// ---- kernel 3: pair gradients and virial; LANES per atom ------------------
// g_ij = dE_i/dr_ij = sum_mu [f_mu'(r) P_mu r_ij / r + f_mu(r) grad P_mu] with
// P_mu = sum_nu dE/dM_{mu,nu} (r_ij)^{(x)nu} (the moment tensors contracted
// with dE/dM); virial S_ab = -sum_j g_a r_b per atom.  G (gradients wanted,
// decided at compile time so that the stores in the pair loop are
// unconditional): the force's own part F_i = sum_j g_ij (FP64, lanes summed
// in a fixed order) is written per atom, and each g_ij is stored at the slot
// of the reverse pair (j, i) -- the gather then subtracts, for every atom,
// the gradients its neighbors hold of it as one contiguous run of its own
// slots, instead of following the reverse index pair by pair.
//
// R > 0 (FP64 only): the rest of the b row in the same pass (kernel 4's
// work, Sec. II.C) -- R = 2 (FULL) the radial-coefficient part
// dV_i/dc_{mu, z_i, z_j, beta} = sum_j T_beta(r_ij) (R_cut - r_ij)^2 P_mu(r_ij)
// from the P_mu and Chebyshev values the gradient already has (32 more FMAs
// per pair at N_rad = 4), then for R = 1 and 2 the species one-hot and the
// zero padding.  The same sums in the same order as kernel 4 at the same
// lanes, so the rows are the same bit for bit.  s_col: the kept-column map
// (R = 2).
template <typename T, int L, int K, bool G, typename TD = T, int R = 0>
__device__ inline void efs_forces_body(const EfsArgs &a, int64_t blk, T *c_s, T (&s_dm)[Level<L>::NC][256 / K],
                                       int32_t *s_col = nullptr) {
    using LV = Level<L>;
    constexpr int NC = LV::NC, NR = LV::NRAD, NL = LV::NLIN;
    constexpr int ND = NR * NPOLY;   // radial-coefficient sums per species (a multiple of K)
    static_assert(R == 0 || sizeof(T) == sizeof(double), "rows are FP64");
    load_coefs<T, NR>(a, c_s);
    const int nt = a.n_types;
    if constexpr (R == 2)   // before load_dm's barrier, which covers it
        for (int k = threadIdx.x; k < NR * nt * nt * NPOLY; k += 256) s_col[k] = a.colmap[nt + NL + k];
    const int sub = threadIdx.x % K;
    const AtomCtx c = atom_ctx<K>(a, blk);
    load_dm<T, NC, K, TD>(a, c, sub, s_dm);
    double *brow = R > 0 && c.live ? a.brow + c.slot : nullptr;   // entry k at brow[k * ldn]
    const int64_t ldn = a.ldn;
    const int la = threadIdx.x / K;
    const T rc = T(a.r_cut);
    const T xs = T(2.0 / (a.r_cut - a.r_min));
    const T x0 = T(-(a.r_min + a.r_cut) / (a.r_cut - a.r_min));
    T vir[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) vir[k] = T(0);
    double fo[3] = {0.0, 0.0, 0.0};   // sum_j g_ij of this lane's pairs
    T *gout = static_cast<T *>(a.gbuf);
    const int32_t *rslot = G ? a.rev + c.atom * (int64_t)a.max_nbrs : nullptr;   // set only with gradients
    int gstart = 0;
    for (int t = 0; t < nt; ++t) {
        const int tc = tcount(a, c, t);
        T dc[R == 2 ? ND : 1];
        if constexpr (R == 2)
#pragma unroll
            for (int k = 0; k < ND; ++k) dc[k] = T(0);
        // the next pair vector is loaded while the current one is used; the
        // loads are unconditional (past the last pair the current one is read
        // again, in bounds and unused), so that the wait for them leaves the
        // gradient stores of the pair before in flight
        const int p0 = gstart + sub < a.max_nbrs ? gstart + sub : a.max_nbrs - 1;
        double nx = c.rp[3 * p0], ny = c.rp[3 * p0 + 1], nz = c.rp[3 * p0 + 2];
        // the reverse slot of the next pair likewise (its store waits for it)
        int nrv = G ? rslot[p0] : 0;
        // waited for here, once, so that the loop head does not wait for
        // every outstanding access (the stores included) on each pair
        __asm__ volatile("" ::"v"(nx), "v"(ny), "v"(nz), "v"(nrv));
        for (int q = sub; q < tc; q += K) {
            const int p = gstart + q;
            const T x = T(nx), y = T(ny), z = T(nz);
            const int rv = nrv;
            const int pn = q + K < tc ? p + K : p;
            nx = c.rp[3 * pn];
            ny = c.rp[3 * pn + 1];
            nz = c.rp[3 * pn + 2];
            if constexpr (G) nrv = rslot[pn];
            const T r = sqrt(x * x + y * y + z * z);
            T g0 = T(0), g1 = T(0), g2 = T(0);
            if (r < rc) {
                T f[NR], fp[NR];
                T qb[R == 2 ? NPOLY : 1];   // T_beta (R_cut - r)^2, for the row's c part
                {
                    const T u = fma(r, xs, x0);
                    const T d = rc - r;
                    const T cut = d * d;
                    const T dcut = T(-2) * d;
                    T Tb[NPOLY], dT[NPOLY];
                    chebyshev<T, true>(u, Tb, dT);
                    if constexpr (R == 2)
#pragma unroll
                        for (int b = 0; b < NPOLY; ++b) qb[b] = Tb[b] * cut;
#pragma unroll
                    for (int mu = 0; mu < NR; ++mu) {
                        const CoefRow<T> cm = coef_row(c_s, mu, c.zi, t, nt);
                        T s = T(0), sp = T(0);
#pragma unroll
                        for (int b = 0; b < NPOLY; ++b) {
                            s = fma(cm[b], Tb[b], s);
                            sp = fma(cm[b], dT[b], sp);
                        }
                        f[mu] = s * cut;
                        fp[mu] = fma(sp * xs, cut, s * dcut);
                    }
                }
                T mono[20];
                efs::monomials(x, y, z, mono);
                T P[NR], Gx[NR], Gy[NR], Gz[NR];
#pragma unroll
                for (int mu = 0; mu < NR; ++mu) P[mu] = Gx[mu] = Gy[mu] = Gz[mu] = T(0);
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const int mu = LV::comp_mu[k];
                    const T dmk = s_dm[k][la];
                    P[mu] = fma(dmk, mono[LV::comp_mono[k]], P[mu]);
                    if (LV::comp_dmonox[k] >= 0)
                        Gx[mu] = fma(dmk * T(LV::comp_dfacx[k]), mono[LV::comp_dmonox[k] < 0 ? 0 : LV::comp_dmonox[k]], Gx[mu]);
                    if (LV::comp_dmonoy[k] >= 0)
                        Gy[mu] = fma(dmk * T(LV::comp_dfacy[k]), mono[LV::comp_dmonoy[k] < 0 ? 0 : LV::comp_dmonoy[k]], Gy[mu]);
                    if (LV::comp_dmonoz[k] >= 0)
                        Gz[mu] = fma(dmk * T(LV::comp_dfacz[k]), mono[LV::comp_dmonoz[k] < 0 ? 0 : LV::comp_dmonoz[k]], Gz[mu]);
                }
                if constexpr (R == 2)
#pragma unroll
                    for (int b = 0; b < NPOLY; ++b)
#pragma unroll
                        for (int mu = 0; mu < NR; ++mu) dc[mu * NPOLY + b] = fma(qb[b], P[mu], dc[mu * NPOLY + b]);
                const T rinv = T(1) / r;
                T radial_part = T(0);
#pragma unroll
                for (int mu = 0; mu < NR; ++mu) {
                    radial_part = fma(fp[mu], P[mu], radial_part);
                    g0 = fma(f[mu], Gx[mu], g0);
                    g1 = fma(f[mu], Gy[mu], g1);
                    g2 = fma(f[mu], Gz[mu], g2);
                }
                radial_part *= rinv;
                g0 = fma(radial_part, x, g0);
                g1 = fma(radial_part, y, g1);
                g2 = fma(radial_part, z, g2);
                // S_ab = -sum g_a r_b
                vir[0] -= g0 * x; vir[1] -= g0 * y; vir[2] -= g0 * z;
                vir[3] -= g1 * x; vir[4] -= g1 * y; vir[5] -= g1 * z;
                vir[6] -= g2 * x; vir[7] -= g2 * y; vir[8] -= g2 * z;
            }
            if constexpr (G) {
                const int64_t s3 = (int64_t)rv * 3;   // the reverse pair's slot
                gout[s3] = g0;
                gout[s3 + 1] = g1;
                gout[s3 + 2] = g2;
                fo[0] += double(g0);
                fo[1] += double(g1);
                fo[2] += double(g2);
            }
        }
        if constexpr (R == 2) {
            efs::reduce_scatter<T, ND, K>(dc, sub);
            if (brow) {
#pragma unroll
                for (int i = 0; i < ND / K; ++i) {
                    const int k = sub * (ND / K) + i, mu = k / NPOLY, b = k % NPOLY;
                    const int col = s_col[((mu * nt + c.zi) * nt + t) * NPOLY + b];
                    if (col >= 0) brow[col * ldn] = dc[i];
                }
            }
        }
        gstart += tc;
    }
    if constexpr (R > 0 && LV::STAGED) {   // (the single-kernel contraction writes these for the other levels)
        if (brow) {   // species one-hot, zero c blocks of the other central species, zero padding
            for (int k = sub; k < nt; k += K) brow[k * ldn] = k == c.zi ? 1.0 : 0.0;
            if constexpr (R == 2) {
                const int nblk = NR * nt * nt * NPOLY;
                for (int k = sub; k < nblk; k += K) {
                    const int zz = (k / (nt * NPOLY)) % nt;
                    if (zz == c.zi) continue;
                    const int col = s_col[k];
                    if (col >= 0) brow[col * ldn] = 0.0;
                }
            }
            for (int k = a.m + sub; k < a.ldb; k += K) brow[k * ldn] = 0.0;
        }
    }
    if constexpr (G) {
#pragma unroll
        for (int o = K / 2; o > 0; o >>= 1)
#pragma unroll
            for (int d = 0; d < 3; ++d) fo[d] += __shfl_xor(fo[d], o, 64);
        if (c.live && sub == 0)
#pragma unroll
            for (int d = 0; d < 3; ++d) a.F[c.atom * 3 + d] = fo[d];
    }
    constexpr int NV = (9 + K - 1) / K * K;
    T vp[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) vp[k] = k < 9 ? vir[k] : T(0);
    efs::reduce_scatter<T, NV, K>(vp, sub);
    if (c.live && a.virial) {
#pragma unroll
        for (int i = 0; i < NV / K; ++i) {
            const int k = sub * (NV / K) + i;
            if (k < 9) a.virial[c.atom * 9 + k] = double(vp[i]);
        }
    }
}

// ---- kernel 4: the rest of b_i (Sec. II.C); LANES per atom ----------------
// FULL grade mode: the radial-coefficient part
//   dV_i/dc_{mu, z_i, z_j, beta} = sum_{j of species z_j} T_beta(r_ij) (R_cut - r_ij)^2 P_mu(r_ij)
// (P_mu as in kernel 3), zero for the blocks of the other central species;
// both modes: the species one-hot (dV_i/dxi0) and zero padding.  The
// xi part (B_alpha) comes from kernel 2.
template <typename T, int L, int K>
__device__ inline void efs_rows_body(const EfsArgs &a, int64_t blk, T (&s_dm)[Level<L>::NC][256 / K],
                                     int32_t *s_col) {
    static_assert(sizeof(T) == sizeof(double), "rows are FP64");
    using LV = Level<L>;
    constexpr int NC = LV::NC, NR = LV::NRAD, NL = LV::NLIN;
    const int nt = a.n_types;
    const int sub = threadIdx.x % K;
    const AtomCtx c = atom_ctx<K>(a, blk);
    const bool full_rows = a.grade_mode == GRADE_FULL;
    if (full_rows) {
        // the kept columns of the c part, once per block in LDS: read from
        // global memory beside the row stores, each would wait for the store
        // before it (the two may alias)
        for (int k = threadIdx.x; k < NR * nt * nt * NPOLY; k += 256) s_col[k] = a.colmap[nt + NL + k];
        load_dm<T, NC, K>(a, c, sub, s_dm);   // (its barrier also covers s_col)
    }
    const int la = threadIdx.x / K;
    // entry k of this neighborhood's row: brow[k * ldn] (column-major rows)
    double *brow = c.live ? a.brow + c.slot : nullptr;
    const int64_t ldn = a.ldn;
    const T rc = T(a.r_cut);
    const T xs = T(2.0 / (a.r_cut - a.r_min));
    const T x0 = T(-(a.r_min + a.r_cut) / (a.r_cut - a.r_min));
    if (full_rows) {
        int gstart = 0;
        for (int t = 0; t < nt; ++t) {
            constexpr int ND = NR * NPOLY;   // a multiple of K (NPOLY = 8)
            T dc[ND];
#pragma unroll
            for (int k = 0; k < ND; ++k) dc[k] = T(0);
            const int tc = tcount(a, c, t);
            double nx = 0.0, ny = 0.0, nz = 0.0;   // next pair vector, in flight
            if (sub < tc) {
                nx = c.rp[3 * (gstart + sub)];
                ny = c.rp[3 * (gstart + sub) + 1];
                nz = c.rp[3 * (gstart + sub) + 2];
            }
            for (int q = sub; q < tc; q += K) {
                const int p = gstart + q;
                const T x = T(nx), y = T(ny), z = T(nz);
                if (q + K < tc) {
                    nx = c.rp[3 * (p + K)];
                    ny = c.rp[3 * (p + K) + 1];
                    nz = c.rp[3 * (p + K) + 2];
                }
                const T r = sqrt(x * x + y * y + z * z);
                if (!(r < rc)) continue;
                const T u = fma(r, xs, x0);
                const T d = rc - r;
                const T cut = d * d;
                T Tb[NPOLY], dT[NPOLY];
                chebyshev<T, false>(u, Tb, dT);
                T mono[20];
                efs::monomials(x, y, z, mono);
                T P[NR];
#pragma unroll
                for (int mu = 0; mu < NR; ++mu) P[mu] = T(0);
#pragma unroll
                for (int k = 0; k < NC; ++k) P[LV::comp_mu[k]] = fma(s_dm[k][la], mono[LV::comp_mono[k]], P[LV::comp_mu[k]]);
#pragma unroll
                for (int b = 0; b < NPOLY; ++b) {
                    const T qb = Tb[b] * cut;
#pragma unroll
                    for (int mu = 0; mu < NR; ++mu) dc[mu * NPOLY + b] = fma(qb, P[mu], dc[mu * NPOLY + b]);
                }
            }
            efs::reduce_scatter<T, ND, K>(dc, sub);
            if (brow) {
#pragma unroll
                for (int i = 0; i < ND / K; ++i) {
                    const int k = sub * (ND / K) + i, mu = k / NPOLY, b = k % NPOLY;
                    const int col = s_col[((mu * nt + c.zi) * nt + t) * NPOLY + b];
                    if (col >= 0) brow[col * ldn] = dc[i];
                }
            }
            gstart += tc;
        }
    }
    if (brow) {
        // species one-hot, zero c blocks of the other central species, zero
        // padding: written here for the staged levels only (the single-kernel
        // contraction writes them for the others)
        if constexpr (Level<L>::STAGED) {
            for (int k = sub; k < nt; k += K) brow[k * ldn] = k == c.zi ? 1.0 : 0.0;
            if (full_rows) {
                const int nblk = NR * nt * nt * NPOLY;
                for (int k = sub; k < nblk; k += K) {
                    const int zz = (k / (nt * NPOLY)) % nt;
                    if (zz == c.zi) continue;
                    const int col = s_col[k];
                    if (col >= 0) brow[col * ldn] = 0.0;
                }
            }
            for (int k = a.m + sub; k < a.ldb; k += K) brow[k * ldn] = 0.0;
        }
    }
}

// Kernels 3 and 4 in one launch: blocks [0, nblk) take kernel 3, blocks
// [nblk, 2 nblk) kernel 4 (when rows are wanted); both only read dE/dM.
// TF: arithmetic of the pair gradients; TD: type of dE/dM, and of the rows
// (rows exist only when TD is FP64: the FP64 form, or the mixed form whose
// contraction ran in FP64 because the grade needs FP64 rows).
template <typename TF, typename TD, int L, int K>
__global__ __launch_bounds__(256) void efs_forces_rows(const EfsArgs a, int64_t nblk) {
    using LV = Level<L>;
    constexpr int NCF = LV::NRAD * MAX_TYPES * MAX_TYPES * NPOLY;
    constexpr size_t FBYTES = sizeof(TF) * (NCF + LV::NC * (256 / K));
    constexpr size_t RBYTES = sizeof(double) * LV::NC * (256 / K) + sizeof(int32_t) * NCF;
    constexpr bool ROWS = sizeof(TD) == sizeof(double);
    // one LDS area: a block takes either the gradient or the row part
    __shared__ __attribute__((aligned(16))) char smem[FBYTES > RBYTES ? FBYTES : RBYTES];
    if ((int64_t)blockIdx.x < nblk) {
        TF *c_s = reinterpret_cast<TF *>(smem);
        auto &s_dm = *reinterpret_cast<TF (*)[LV::NC][256 / K]>(c_s + NCF);
        if (a.gbuf)
            efs_forces_body<TF, L, K, true, TD>(a, blockIdx.x, c_s, s_dm);
        else
            efs_forces_body<TF, L, K, false, TD>(a, blockIdx.x, c_s, s_dm);
        if (a.part) {   // uniform: the block's atoms are whole sum chunks (256 / K = 32, 64 or 128)
            constexpr int PER = 256 / K / SUM_CHUNK;
            static_assert(PER * SUM_CHUNK * K == 256, "chunks per block");
            for (int q = 0; q < PER; ++q) {
                const int64_t chunk = (int64_t)blockIdx.x * PER + q;
                __syncthreads();   // the block's virials are written; sp of the previous chunk is read
                if (chunk * SUM_CHUNK < a.n_atoms) chunk_partials(chunk, a.n_atoms, a.part_e, a.virial, a.part);
            }
        }
    } else if constexpr (ROWS) {
        auto &s_dm = *reinterpret_cast<double (*)[LV::NC][256 / K]>(smem);
        int32_t *s_col = reinterpret_cast<int32_t *>(smem + sizeof(double) * LV::NC * (256 / K));
        efs_rows_body<double, L, K>(a, (int64_t)blockIdx.x - nblk, s_dm, s_col);
    }
}

// FP64 form with forces and rows: kernels 3 and 4 in one pass over the pairs
// (R = 1 LINEAR, 2 FULL rows); no row blocks
template <typename T, int L, int K, int R>
__global__ __launch_bounds__(256) void efs_forces_fused(const EfsArgs a) {
    using LV = Level<L>;
    constexpr int NCF = LV::NRAD * MAX_TYPES * MAX_TYPES * NPOLY;
    __shared__ __attribute__((aligned(16))) char smem[sizeof(T) * (NCF + LV::NC * (256 / K)) + sizeof(int32_t) * NCF];
    T *c_s = reinterpret_cast<T *>(smem);
    auto &s_dm = *reinterpret_cast<T (*)[LV::NC][256 / K]>(c_s + NCF);
    int32_t *s_col = reinterpret_cast<int32_t *>(smem + sizeof(T) * (NCF + LV::NC * (256 / K)));
    efs_forces_body<T, L, K, true, T, R>(a, blockIdx.x, c_s, s_dm, s_col);
    if (a.part) {   // uniform: the block's atoms are whole sum chunks
        constexpr int PER = 256 / K / SUM_CHUNK;
        static_assert(PER * SUM_CHUNK * K == 256, "chunks per block");
        for (int q = 0; q < PER; ++q) {
            const int64_t chunk = (int64_t)blockIdx.x * PER + q;
            __syncthreads();
            if (chunk * SUM_CHUNK < a.n_atoms) chunk_partials(chunk, a.n_atoms, a.part_e, a.virial, a.part);
        }
    }
}

template <int L, typename T> int launch_mc_level_t(const EfsArgs &a);
template <int L, typename TF, typename TD> int launch_fr_level_t(const EfsArgs &a);

// instantiates the launchers of one level and one arithmetic type (each
// (level, type) pair is a translation unit of its own, generated at build
// time): the moments / contraction in TT (rows only when TT is FP64), the
// pair gradients in TT with dE/dM in TT, and for TT = float also with dE/dM
// in FP64 (the mixed form with FP64 rows)
#define MTP_EFS_MC_LEVEL_T(LEVEL, TT)                                                                    \
    /* moments and contraction, K lanes per neighborhood (K = 4, 8: one launch; K = 2: two) */         \
    template <typename T, int K, bool WB> static void launch_mc##LEVEL(const EfsArgs &a) {               \
        const unsigned grid = (unsigned)((a.n_atoms + 256 / K - 1) / (256 / K));                         \
        const unsigned grid1 = (unsigned)((a.n_atoms + 63) / 64);                                        \
        if (K == 4) {                                                                                    \
            ProfScope ps("efs_moments", a.stream);                                                       \
            hipLaunchKernelGGL((efs_moments_contract<T, LEVEL, WB>), dim3(grid1), dim3(256), 0, a.stream, \
                               a);                                                                       \
        } else if (K == 8) {                                                                             \
            ProfScope ps("efs_moments", a.stream);                                                       \
            hipLaunchKernelGGL((efs_moments_contract8<T, LEVEL, WB>), dim3(grid1), dim3(512), 0,          \
                               a.stream, a);                                                             \
        } else {                                                                                         \
            {                                                                                            \
                ProfScope ps("efs_moments", a.stream);                                                   \
                hipLaunchKernelGGL((efs_moments<T, LEVEL, K>), dim3(grid), dim3(256), 0, a.stream, a);   \
            }                                                                                            \
            ProfScope ps("efs_contract", a.stream);                                                      \
            hipLaunchKernelGGL((efs_contract<T, LEVEL, WB>), dim3(grid1), dim3(256), 0, a.stream, a);    \
        }                                                                                                \
    }                                                                                                    \
    template <> int launch_mc_level_t<LEVEL, TT>(const EfsArgs &a) {                                     \
        if (a.n_atoms == 0) return 0;                                                                    \
        constexpr bool F64 = sizeof(TT) == sizeof(double);                                               \
        if (F64 && a.brow != nullptr) {                                                                  \
            switch (a.lanes_mc) {                                                                        \
                case 2: launch_mc##LEVEL<TT, 2, F64>(a); break;                                          \
                case 4: launch_mc##LEVEL<TT, 4, F64>(a); break;                                          \
                default: launch_mc##LEVEL<TT, 8, F64>(a); break;                                         \
            }                                                                                            \
        } else {                                                                                         \
            switch (a.lanes_mc) {                                                                        \
                case 2: launch_mc##LEVEL<TT, 2, false>(a); break;                                        \
                case 4: launch_mc##LEVEL<TT, 4, false>(a); break;                                        \
                default: launch_mc##LEVEL<TT, 8, false>(a); break;                                       \
            }                                                                                            \
        }                                                                                                \
        return (int)hipGetLastError();                                                                   \
    }

#define MTP_EFS_FR_LEVEL_T(LEVEL, TT)                                                                    \
    /* pair gradients and virial (+ the rest of the rows), K lanes per neighborhood */                   \
    template <typename TF, typename TD, int K> static void launch_fr##LEVEL(const EfsArgs &a) {          \
        const unsigned grid = (unsigned)((a.n_atoms + 256 / K - 1) / (256 / K));                         \
        const bool rows = sizeof(TD) == sizeof(double) && a.brow != nullptr;                             \
        ProfScope ps("efs_forces", a.stream);                                                            \
        if constexpr (sizeof(TF) == sizeof(double)) {                                                    \
            if (rows && a.gbuf) { /* FP64 with forces: rows in the same pass */                          \
                if (a.grade_mode == GRADE_FULL)                                                          \
                    hipLaunchKernelGGL((efs_forces_fused<TF, LEVEL, K, 2>), dim3(grid), dim3(256), 0,     \
                                       a.stream, a);                                                     \
                else                                                                                     \
                    hipLaunchKernelGGL((efs_forces_fused<TF, LEVEL, K, 1>), dim3(grid), dim3(256), 0,     \
                                       a.stream, a);                                                     \
                return;                                                                                  \
            }                                                                                            \
        }                                                                                                \
        hipLaunchKernelGGL((efs_forces_rows<TF, TD, LEVEL, K>), dim3(rows ? 2 * grid : grid), dim3(256),  \
                           0, a.stream, a, (int64_t)grid);                                               \
    }                                                                                                    \
    template <typename TD> static int launch_fr_td##LEVEL(const EfsArgs &a) {                            \
        if (a.n_atoms == 0) return 0;                                                                    \
        switch (a.lanes) {                                                                               \
            case 2: launch_fr##LEVEL<TT, TD, 2>(a); break;                                               \
            case 4: launch_fr##LEVEL<TT, TD, 4>(a); break;                                               \
            default: launch_fr##LEVEL<TT, TD, 8>(a); break;                                              \
        }                                                                                                \
        return (int)hipGetLastError();                                                                   \
    }                                                                                                    \
    template <> int launch_fr_level_t<LEVEL, TT, TT>(const EfsArgs &a) { return launch_fr_td##LEVEL<TT>(a); } \
    MTP_EFS_HYBRID_##TT(LEVEL)

#define MTP_EFS_HYBRID_double(LEVEL)
#define MTP_EFS_HYBRID_float(LEVEL)                                                                      \
    template <> int launch_fr_level_t<LEVEL, float, double>(const EfsArgs &a) {                          \
        return launch_fr_td##LEVEL<double>(a);                                                           \
    }

}  // namespace mtp
