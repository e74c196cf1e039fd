// Gradient of the fitting objective (MLIP-3 paper eq. 7) with respect to
// theta, given the upstream gradients gE = dL/dE, gF = dL/dF, gS = dL/dS.
//
// Because F = -dE/dx and S = -dE/deps, the force and stress terms are
// -d/dtheta of one directional derivative of E: along x -> x + t gF and
// eps = t gS every pair vector moves by
//     dr_ij = gF_j - gF_i + gS r_ij,
// and dE/dt = sum_i dV_i/dt with dV_i/dt = sum_j g_ij . dr_ij.  So
//     dL/dtheta = sum_i [ gE_cfg(i) dV_i/dtheta - d(dV_i/dt)/dtheta ].
// Per neighborhood (moments recomputed, nothing stored per pair):
//   * tangent moments  Mdot_k = sum_j d(f_mu m_k)/dr . dr_ij;
//   * the contraction program run on dual numbers (value, tangent) gives
//     B_alpha and Bdot_alpha, dV/dM and its tangent H Mdot;
//   * theta = xi_alpha:   gE B_alpha - Bdot_alpha;  theta = xi_0[z_i]: gE;
//   * theta = c^(beta)_{mu,z_i,z}: sum over pairs with z_j = z of
//       gE Q_beta P_mu - [ Q_beta (Phat_mu + grad P_mu . dr) + Q'_beta (rhat . dr) P_mu ]
//     with P_mu = sum_{k in mu} (dV/dM_k) m_k and Phat_mu the same with H Mdot.
// Each neighborhood writes its row of contributions; a column reduction in
// FP64 adds the rows in a fixed order.
#pragma once

#include "efs_kernel.hpp"

namespace mtp {
namespace ad {   // dual numbers; fma for them is found by argument-dependent lookup

template <typename T> struct Dual {
    T v, d;
    Dual() = default;
    __device__ constexpr Dual(T x) : v(x), d(T(0)) {}
    __device__ constexpr Dual(T x, T y) : v(x), d(y) {}
    __device__ Dual &operator+=(const Dual &o) {
        v += o.v;
        d += o.d;
        return *this;
    }
};
template <typename T> __device__ inline Dual<T> operator*(const Dual<T> &a, const Dual<T> &b) {
    return Dual<T>(a.v * b.v, ::fma(a.v, b.d, a.d * b.v));
}
template <typename T> __device__ inline Dual<T> operator+(const Dual<T> &a, const Dual<T> &b) {
    return Dual<T>(a.v + b.v, a.d + b.d);
}
template <typename T> __device__ inline Dual<T> fma(const Dual<T> &a, const Dual<T> &b, const Dual<T> &c) {
    return Dual<T>(::fma(a.v, b.v, c.v), ::fma(a.v, b.d, ::fma(a.d, b.v, c.d)));
}

}  // namespace ad
using ad::Dual;

// xi as constants of the dual program
template <typename T> struct XiConst {
    const T *p;
    __device__ Dual<T> operator[](int a) const { return Dual<T>(p[a]); }
};

// receives B_alpha (value, tangent) and writes gE B - Bdot into the row
template <typename T> struct GradSink {
    T *row;
    T gE;
    struct Ref {
        T *p;
        T gE;
        __device__ void operator=(const Dual<T> &b) const { *p = fma(gE, b.v, -b.d); }
    };
    __device__ Ref operator[](int a) const { return Ref{row + a, gE}; }
};


template <typename T> __device__ inline void pair_dr(const BwdArgs &b, int64_t atom, int64_t slot, T x, T y, T z,
                                                     T &d0, T &d1, T &d2) {
    d0 = d1 = d2 = T(0);
    if (b.gF) {
        const int j = b.nbr_j[slot];
        d0 = T(b.gF[3 * j] - b.gF[3 * atom]);
        d1 = T(b.gF[3 * j + 1] - b.gF[3 * atom + 1]);
        d2 = T(b.gF[3 * j + 2] - b.gF[3 * atom + 2]);
    }
    if (b.gS) {
        const double *W = b.gS + 9 * (int64_t)b.atom_cfg[atom];
        d0 = fma(T(W[0]), x, fma(T(W[1]), y, fma(T(W[2]), z, d0)));
        d1 = fma(T(W[3]), x, fma(T(W[4]), y, fma(T(W[5]), z, d1)));
        d2 = fma(T(W[6]), x, fma(T(W[7]), y, fma(T(W[8]), z, d2)));
    }
}

// ---- tangent moments ------------------------------------------------------
template <typename T, int L, int K>
__global__ __launch_bounds__(256) void bwd_tangent_moments(const BwdArgs b) {
    using LV = Level<L>;
    constexpr int NC = LV::NC, NR = LV::NRAD;
    const EfsArgs &a = b.e;
    __shared__ T c_s[NR * MAX_TYPES * MAX_TYPES * NPOLY];
    load_coefs<T, NR>(a, c_s);
    const int nt = a.n_types;
    const int sub = threadIdx.x % K;
    const AtomCtx c = atom_ctx<K>(a);
    const T rc = T(a.r_cut);
    const T xs = T(2.0 / (a.r_cut - a.r_min));
    const T x0 = T(-(a.r_min + a.r_cut) / (a.r_cut - a.r_min));
    T Md[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) Md[k] = T(0);
    int zj = 0, tend = c.tc[0];
    for (int p = sub; p < c.ntot; p += K) {
        while (p >= tend && zj < nt - 1) tend += c.tc[++zj];
        const T x = T(c.rp[3 * p]), y = T(c.rp[3 * p + 1]), z = T(c.rp[3 * p + 2]);
        const T r = sqrt(x * x + y * y + z * z);
        if (!(r < rc)) continue;
        T d0, d1, d2;
        pair_dr<T>(b, c.atom, c.atom * (int64_t)a.max_nbrs + p, x, y, z, d0, d1, d2);
        const T rdot = (x * d0 + y * d1 + z * d2) / r;
        T f[NR], fp[NR];
        {
            const T u = fma(r, xs, x0), dd = rc - r, cut = dd * dd, dcut = T(-2) * dd;
            T Tb[NPOLY], dT[NPOLY];
            Tb[0] = T(1);
            Tb[1] = u;
            dT[0] = T(0);
            dT[1] = T(1);
#pragma unroll
            for (int q = 2; q < NPOLY; ++q) {
                Tb[q] = fma(T(2) * u, Tb[q - 1], -Tb[q - 2]);
                dT[q] = fma(T(2) * u, dT[q - 1], fma(T(2), Tb[q - 1], -dT[q - 2]));
            }
#pragma unroll
            for (int mu = 0; mu < NR; ++mu) {
                const CoefRow<T> cm = coef_row(c_s, mu, c.zi, zj, nt);
                T s = T(0), sp = T(0);
#pragma unroll
                for (int q = 0; q < NPOLY; ++q) {
                    s = fma(cm[q], Tb[q], s);
                    sp = fma(cm[q], dT[q], sp);
                }
                f[mu] = s * cut;
                fp[mu] = fma(sp * xs, cut, s * dcut);
            }
        }
        T mono[20];
        efs::monomials(x, y, z, mono);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int mu = LV::comp_mu[k];
            T gdot = T(0);
            if (LV::comp_dmonox[k] >= 0)
                gdot = fma(T(LV::comp_dfacx[k]) * mono[LV::comp_dmonox[k] < 0 ? 0 : LV::comp_dmonox[k]], d0, gdot);
            if (LV::comp_dmonoy[k] >= 0)
                gdot = fma(T(LV::comp_dfacy[k]) * mono[LV::comp_dmonoy[k] < 0 ? 0 : LV::comp_dmonoy[k]], d1, gdot);
            if (LV::comp_dmonoz[k] >= 0)
                gdot = fma(T(LV::comp_dfacz[k]) * mono[LV::comp_dmonoz[k] < 0 ? 0 : LV::comp_dmonoz[k]], d2, gdot);
            Md[k] = fma(fp[mu] * rdot, mono[LV::comp_mono[k]], fma(f[mu], gdot, Md[k]));
        }
    }
#pragma unroll
    for (int o = K / 2; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < NC; ++k) Md[k] += efs::xor_shuffle(Md[k], o);
    if (c.live) {
        T *out = static_cast<T *>(b.tbuf);
#pragma unroll
        for (int k = 0; k < NC; ++k)
            if (k % K == sub) out[(int64_t)k * a.n_atoms + c.slot] = Md[k];
    }
}

// ---- dual contraction -------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(256) void bwd_contract(const BwdArgs b) {
    using LV = Level<L>;
    constexpr int NC = LV::NC;
    const EfsArgs &a = b.e;
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= a.n_atoms) return;
    const int nt = a.n_types;
    const T *mv = static_cast<const T *>(a.mbuf);
    const T *mt = static_cast<const T *>(b.tbuf);
    Dual<T> M[NC], dM[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) M[k] = Dual<T>(mv[(int64_t)k * a.n_atoms + slot], mt[(int64_t)k * a.n_atoms + slot]);
    Dual<T> V(T(0));
    int zi = a.type[slot];
    zi = zi < 0 ? 0 : (zi >= nt ? nt - 1 : zi);
    const T gE = b.gE ? T(b.gE[b.atom_cfg[slot]]) : T(0);
    T *row = static_cast<T *>(b.rows) + slot * (int64_t)b.n_theta;
    for (int t = 0; t < nt; ++t) row[t] = t == zi ? gE : T(0);
    LV::template contract<Dual<T>, true>(M, XiConst<T>{xi_of<T>(a)}, GradSink<T>{row + nt, gE}, dM,
                                         V);
    T *dv = static_cast<T *>(a.dmbuf);
    T *dt = static_cast<T *>(b.dtbuf);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        dv[(int64_t)k * a.n_atoms + slot] = dM[k].v;
        dt[(int64_t)k * a.n_atoms + slot] = dM[k].d;
    }
}

// ---- c part of the rows -----------------------------------------------------
template <typename T, int L, int K>
__global__ __launch_bounds__(256) void bwd_pairs(const BwdArgs b) {
    using LV = Level<L>;
    constexpr int NC = LV::NC, NR = LV::NRAD, NL = LV::NLIN;
    const EfsArgs &a = b.e;
    __shared__ T c_s[NR * MAX_TYPES * MAX_TYPES * NPOLY];
    load_coefs<T, NR>(a, c_s);
    const int nt = a.n_types;
    const int sub = threadIdx.x % K;
    const AtomCtx c = atom_ctx<K>(a);
    const T rc = T(a.r_cut);
    const T xs = T(2.0 / (a.r_cut - a.r_min));
    const T x0 = T(-(a.r_min + a.r_cut) / (a.r_cut - a.r_min));
    T dv[NC], dt[NC];
    {
        const T *pv = static_cast<const T *>(a.dmbuf);
        const T *pt = static_cast<const T *>(b.dtbuf);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            dv[k] = c.live ? pv[(int64_t)k * a.n_atoms + c.slot] : T(0);
            dt[k] = c.live ? pt[(int64_t)k * a.n_atoms + c.slot] : T(0);
        }
    }
    const T gE = (c.live && b.gE) ? T(b.gE[b.atom_cfg[c.atom]]) : T(0);
    T *row = c.live ? static_cast<T *>(b.rows) + c.slot * (int64_t)b.n_theta + nt + NL : nullptr;
    int gstart = 0;
    for (int t = 0; t < nt; ++t) {
        T acc[NR][NPOLY];
#pragma unroll
        for (int mu = 0; mu < NR; ++mu)
#pragma unroll
            for (int q = 0; q < NPOLY; ++q) acc[mu][q] = T(0);
        for (int qq = sub; qq < tcount(a, c, t); qq += K) {
            const int p = gstart + qq;
            const T x = T(c.rp[3 * p]), y = T(c.rp[3 * p + 1]), z = T(c.rp[3 * p + 2]);
            const T r = sqrt(x * x + y * y + z * z);
            if (!(r < rc)) continue;
            T d0, d1, d2;
            pair_dr<T>(b, c.atom, c.atom * (int64_t)a.max_nbrs + p, x, y, z, d0, d1, d2);
            const T rdot = (x * d0 + y * d1 + z * d2) / r;
            T Q[NPOLY], Qp[NPOLY];
            {
                const T u = fma(r, xs, x0), dd = rc - r, cut = dd * dd, dcut = T(-2) * dd;
                T Tb[NPOLY], dT[NPOLY];
                Tb[0] = T(1);
                Tb[1] = u;
                dT[0] = T(0);
                dT[1] = T(1);
#pragma unroll
                for (int q = 2; q < NPOLY; ++q) {
                    Tb[q] = fma(T(2) * u, Tb[q - 1], -Tb[q - 2]);
                    dT[q] = fma(T(2) * u, dT[q - 1], fma(T(2), Tb[q - 1], -dT[q - 2]));
                }
#pragma unroll
                for (int q = 0; q < NPOLY; ++q) {
                    Q[q] = Tb[q] * cut;
                    Qp[q] = fma(dT[q] * xs, cut, Tb[q] * dcut);
                }
            }
            T mono[20];
            efs::monomials(x, y, z, mono);
            T P[NR], Ph[NR], GP[NR];
#pragma unroll
            for (int mu = 0; mu < NR; ++mu) P[mu] = Ph[mu] = GP[mu] = T(0);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int mu = LV::comp_mu[k];
                const T m = mono[LV::comp_mono[k]];
                P[mu] = fma(dv[k], m, P[mu]);
                Ph[mu] = fma(dt[k], m, Ph[mu]);
                T gdot = T(0);
                if (LV::comp_dmonox[k] >= 0)
                    gdot = fma(T(LV::comp_dfacx[k]) * mono[LV::comp_dmonox[k] < 0 ? 0 : LV::comp_dmonox[k]], d0, gdot);
                if (LV::comp_dmonoy[k] >= 0)
                    gdot = fma(T(LV::comp_dfacy[k]) * mono[LV::comp_dmonoy[k] < 0 ? 0 : LV::comp_dmonoy[k]], d1, gdot);
                if (LV::comp_dmonoz[k] >= 0)
                    gdot = fma(T(LV::comp_dfacz[k]) * mono[LV::comp_dmonoz[k] < 0 ? 0 : LV::comp_dmonoz[k]], d2, gdot);
                GP[mu] = fma(dv[k], gdot, GP[mu]);
            }
#pragma unroll
            for (int mu = 0; mu < NR; ++mu) {
                const T w1 = fma(gE, P[mu], -(Ph[mu] + GP[mu]));   // multiplies Q_beta
                const T w2 = -rdot * P[mu];                         // multiplies Q'_beta
#pragma unroll
                for (int q = 0; q < NPOLY; ++q) acc[mu][q] = fma(w1, Q[q], fma(w2, Qp[q], acc[mu][q]));
            }
        }
#pragma unroll
        for (int o = K / 2; o > 0; o >>= 1)
#pragma unroll
            for (int mu = 0; mu < NR; ++mu)
#pragma unroll
                for (int q = 0; q < NPOLY; ++q) acc[mu][q] += efs::xor_shuffle(acc[mu][q], o);
        if (row) {
#pragma unroll
            for (int mu = 0; mu < NR; ++mu)
#pragma unroll
                for (int q = 0; q < NPOLY; ++q)
                    if ((mu * NPOLY + q) % K == sub) row[((mu * nt + c.zi) * nt + t) * NPOLY + q] = acc[mu][q];
        }
        gstart += tcount(a, c, t);
    }
    if (row) {   // c blocks of the other central species are zero
        const int nblk = NR * nt * nt * NPOLY;
        for (int k = sub; k < nblk; k += K)
            if ((k / (nt * NPOLY)) % nt != c.zi) row[k] = T(0);
    }
}

template <int L, typename T> int launch_backward_level_t(const BwdArgs &b);

#define MTP_BWD_LEVEL_T(LEVEL, TT)                                                                        \
    template <typename T, int K> static void launch_bwd_tk##LEVEL(const BwdArgs &b) {                     \
        const int per = 256 / K;                                                                          \
        const unsigned grid = (unsigned)((b.e.n_atoms + per - 1) / per);                                  \
        const unsigned grid1 = (unsigned)((b.e.n_atoms + 255) / 256);                                     \
        if (grid == 0) return;                                                                            \
        hipLaunchKernelGGL((efs_moments<T, LEVEL, K>), dim3(grid), dim3(256), 0, b.e.stream, b.e);        \
        hipLaunchKernelGGL((bwd_tangent_moments<T, LEVEL, K>), dim3(grid), dim3(256), 0, b.e.stream, b);  \
        hipLaunchKernelGGL((bwd_contract<T, LEVEL>), dim3(grid1), dim3(256), 0, b.e.stream, b);           \
        hipLaunchKernelGGL((bwd_pairs<T, LEVEL, K>), dim3(grid), dim3(256), 0, b.e.stream, b);            \
    }                                                                                                     \
    template <> int launch_backward_level_t<LEVEL, TT>(const BwdArgs &b) {                                \
        launch_bwd_tk##LEVEL<TT, 4>(b);                                                                   \
        return (int)hipGetLastError();                                                                    \
    }

}  // namespace mtp
