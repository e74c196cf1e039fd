// Staged contraction for the levels whose program is too large for one
// kernel (level 24: 218 connected graphs, 941 basis functions, about 294 k
// flops per neighborhood).  The single-kernel contraction holds every graph
// value and dV/dg of a neighborhood in registers and exchanges the graph
// values of 64 neighborhoods through LDS; at this level that is 2 x 218
// values per lane and 111 KB of LDS (FP64), beyond a CU.  Here the program
// runs as separate launches that pass per-neighborhood state through memory:
//
//   moments (efs_moments)          -> M      [NC][n]
//   graph values, part P of 8      -> g      tiles of 64 neighborhoods (reads M)
//   trie walk                      -> dV/dg  tiles; V; B_alpha rows
//   reverse pass, part P of 16     -> dV/dM  [NC][n]       (reads M, dV/dg;
//                                     part P adds its share to parts 0..P-1)
//
// followed by the pair-gradient kernel as at every level.  One neighborhood
// per lane throughout.  The graphs of a part are chosen so that they use few
// moment components (the generator clusters them), which the part holds in
// registers; each part is its own translation unit, so the program compiles
// in pieces.  The state is about 4 KB per neighborhood (FP64): a few GB of
// HBM traffic per 10^6 atoms.
#pragma once

#include "efs_kernel.hpp"

namespace mtp {

// in the trie walk, after the nodes of the first two depths: dV/dg goes back
// to memory and the graph values are read again (a compiler barrier), and
// the running sum w of the parent node is formed there (else its products
// are deferred to the end, every factor held until then); deeper nodes only
// pin w (MTP_STAGE_KEEP)
#define MTP_STAGE_SYNC(w) asm volatile("" : "+v"(w) : : "memory")
// a Horner sum formed where it is written (not deferred)
#define MTP_STAGE_KEEP(a) asm volatile("" : "+v"(a))

// between the graphs of a part: no instruction is scheduled across, so that
// the graphs are not interleaved (which would hold the temporaries of many at
// once on top of the part's moments and dV/dM)
#define MTP_STAGE_SCHED() __builtin_amdgcn_sched_barrier(0)

template <int L, int P> struct LevelGraphs;
template <int L, int P> struct LevelReverse;

// Graph values and dV/dg are stored in tiles of 64 neighborhoods,
// [n / 64][NGRAPH][64]: the tile base is uniform over a wavefront (scalar
// registers) and the lane's offset is one vector register, so the thousands
// of accesses of the trie walk need no per-access 64-bit vector address.
template <typename T> struct TileCol {
    T *base;         // this wavefront's tile
    uint32_t lane;
    __device__ T &operator[](int k) const { return base[k * 64 + lane]; }
};
template <typename T, int NG> __device__ inline TileCol<T> tile_of(T *arr, int64_t slot) {
    const int64_t tile = __builtin_amdgcn_readfirstlane((int)(slot >> 6));   // uniform: 64 slots per wavefront
    return TileCol<T>{arr + tile * (int64_t)NG * 64, (uint32_t)(slot & 63)};
}

// the moment components a part uses, from memory into registers (the
// others are never read)
template <typename T, typename PART, int NC>
__device__ inline void load_part_moments(const EfsArgs &a, int64_t slot, T (&M)[NC]) {
    const T *mb = static_cast<const T *>(a.mbuf) + slot;
#pragma unroll
    for (int i = 0; i < PART::NM; ++i) M[PART::mcomp[i]] = mb[(int64_t)PART::mcomp[i] * a.n_atoms];
}

template <typename T, int L, int P>
__global__ __launch_bounds__(256) void efs_graphs_stage(const EfsArgs a) {
    using LV = Level<L>;
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= a.n_atoms) return;
    T M[LV::NC];
    load_part_moments<T, LevelGraphs<L, P>>(a, slot, M);
    LevelGraphs<L, P>::template run<T>(M, tile_of<T, LV::NGRAPH>(static_cast<T *>(a.gval), slot));
}

template <typename T, int L, bool WB>
__global__ __launch_bounds__(256) void efs_trie_stage(const EfsArgs a, const T *__restrict__ gval,
                                                     T *__restrict__ dgval) {
    using LV = Level<L>;
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= a.n_atoms) return;
    const TileCol<const T> gin = tile_of<const T, LV::NGRAPH>(gval, slot);
    const TileCol<T> dg = tile_of<T, LV::NGRAPH>(dgval, slot);
    const XiPtr<T> xi{xi_of<T>(a)};
    T V = T(0);
    if constexpr (WB) {
        static_assert(sizeof(T) == sizeof(double), "rows are FP64");
        LV::template trie<T, true>(gin, xi, ColSink{a.brow, a.ldn, a.n_types, (uint32_t)slot, true}, dg, V);
    } else {
        LV::template trie<T, false>(gin, xi, NoSink{}, dg, V);
    }
    if (a.site_e) {
        const int64_t atom = a.atom_list ? (int64_t)a.atom_list[slot] : slot;
        int zi = a.type[atom];
        zi = zi < 0 ? 0 : (zi >= a.n_types ? a.n_types - 1 : zi);
        a.site_e[atom] = double(V) + double(xi0_of<T>(a)[zi]);
    }
}

template <typename T, int L, int P>
__global__ __launch_bounds__(256, 2) void efs_reverse_stage(const EfsArgs a) {
    using LV = Level<L>;
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= a.n_atoms) return;
    using PART = LevelReverse<L, P>;
    T M[LV::NC], dM[LV::NC];
    load_part_moments<T, PART>(a, slot, M);
    PART::template run<T>(M, tile_of<const T, LV::NGRAPH>(static_cast<const T *>(a.dgval), slot), dM);
    T *out = static_cast<T *>(a.dmbuf) + slot;
    if constexpr (P == 0) {   // part 0 writes every component (zero where it adds nothing)
#pragma unroll
        for (int k = 0; k < LV::NC; ++k) out[(int64_t)k * a.n_atoms] = dM[k];
    } else {                  // the others add to theirs, in part order: deterministic
#pragma unroll
        for (int i = 0; i < PART::NM; ++i) {
            const int64_t o = (int64_t)PART::mcomp[i] * a.n_atoms;
            out[o] = out[o] + dM[PART::mcomp[i]];
        }
    }
}

template <int L, typename T, int P> void launch_graphs_stage(const EfsArgs &a);
template <int L, typename T, int P> void launch_reverse_stage(const EfsArgs &a);

// one unit per graph part / reverse part (and arithmetic type)
#define MTP_STAGE_G_T(LEVEL, TT, P)                                                                      \
    template <> void launch_graphs_stage<LEVEL, TT, P>(const EfsArgs &a) {                               \
        hipLaunchKernelGGL((efs_graphs_stage<TT, LEVEL, P>), dim3((unsigned)((a.n_atoms + 255) / 256)),  \
                           dim3(256), 0, a.stream, a);                                                   \
    }
#define MTP_STAGE_R_T(LEVEL, TT, P)                                                                      \
    template <> void launch_reverse_stage<LEVEL, TT, P>(const EfsArgs &a) {                              \
        hipLaunchKernelGGL((efs_reverse_stage<TT, LEVEL, P>), dim3((unsigned)((a.n_atoms + 255) / 256)), \
                           dim3(256), 0, a.stream, a);                                                   \
    }

template <int L, typename T, int... P>
static void launch_stages(const EfsArgs &a, std::integer_sequence<int, P...>, bool graphs) {
    if (graphs)
        (launch_graphs_stage<L, T, P>(a), ...);
    else
        (launch_reverse_stage<L, T, P>(a), ...);
}

// the moments / contraction launcher of a staged level (the pair-gradient
// launcher is the common one)
#define MTP_EFS_STAGED_LEVEL_T(LEVEL, TT)                                                                \
    template <> int launch_mc_level_t<LEVEL, TT>(const EfsArgs &a) {                                     \
        using LV = Level<LEVEL>;                                                                         \
        if (a.n_atoms == 0) return 0;                                                                    \
        constexpr bool F64 = sizeof(TT) == sizeof(double);                                               \
        const unsigned g256 = (unsigned)((a.n_atoms + 255) / 256);                                       \
        {                                                                                                \
            ProfScope ps("efs_moments", a.stream);                                                       \
            const int K = a.lanes_mc == 2 ? 2 : (a.lanes_mc == 4 ? 4 : 8);                               \
            const unsigned grid = (unsigned)((a.n_atoms + 256 / K - 1) / (256 / K));                     \
            if (K == 2)                                                                                  \
                hipLaunchKernelGGL((efs_moments<TT, LEVEL, 2>), dim3(grid), dim3(256), 0, a.stream, a);  \
            else if (K == 4)                                                                             \
                hipLaunchKernelGGL((efs_moments<TT, LEVEL, 4>), dim3(grid), dim3(256), 0, a.stream, a);  \
            else                                                                                         \
                hipLaunchKernelGGL((efs_moments<TT, LEVEL, 8>), dim3(grid), dim3(256), 0, a.stream, a);  \
        }                                                                                                \
        ProfScope ps("efs_contract", a.stream);                                                          \
        launch_stages<LEVEL, TT>(a, std::make_integer_sequence<int, LV::STAGE_G>{}, true);               \
        const TT *gv = static_cast<const TT *>(a.gval);                                                   \
        TT *dgv = static_cast<TT *>(a.dgval);                                                            \
        if (F64 && a.brow != nullptr)                                                                    \
            hipLaunchKernelGGL((efs_trie_stage<TT, LEVEL, F64>), dim3(g256), dim3(256), 0, a.stream, a, gv, \
                               dgv);                                                                     \
        else                                                                                             \
            hipLaunchKernelGGL((efs_trie_stage<TT, LEVEL, false>), dim3(g256), dim3(256), 0, a.stream, a, gv, \
                               dgv);                                                                     \
        launch_stages<LEVEL, TT>(a, std::make_integer_sequence<int, LV::STAGE_R>{}, false);              \
        return (int)hipGetLastError();                                                                   \
    }

}  // namespace mtp
