// Host build of the generated contraction programs (device qualifiers and the
// staged form's compiler barriers defined away): the staged program of a
// level (graph values in Horner form, streamed trie walk, reverse pass in
// parts) against the single-kernel program of the same level, on random
// moments and xi.  Built and run by tests/test_generator_forms.py.
#include <cmath>
#include <cstdio>
#include <random>
#define __device__
#define __forceinline__ inline
#define MTP_STAGE_SYNC(w)
#define MTP_STAGE_SCHED()
#define MTP_STAGE_KEEP(a)
using std::fma;
namespace A {
template <int L> struct Level;
#include LEVEL_A
}
namespace B {
template <int L> struct Level;
template <int L, int P> struct LevelGraphs;
template <int L, int P> struct LevelReverse;
#include LEVEL_B
#include "parts.inc"
}
template <int P> void graphs(const double *M, double *G) {
    if constexpr (P < B::Level<LV>::STAGE_G) { B::LevelGraphs<LV, P>::template run<double>(M, G); graphs<P + 1>(M, G); }
}
template <int P> void reverse(const double *M, const double *dg, double *dM) {
    if constexpr (P < B::Level<LV>::STAGE_R) {
        double d[B::Level<LV>::NC];
        B::LevelReverse<LV, P>::template run<double>(M, dg, d);
        for (int k = 0; k < B::Level<LV>::NC; ++k) dM[k] += d[k];
        reverse<P + 1>(M, dg, dM);
    }
}
int main() {
    using LA = A::Level<LV>;
    using LB = B::Level<LV>;
    constexpr int NC = LA::NC, NL = LA::NLIN, NG = LA::NGRAPH;
    std::mt19937_64 rng(5);
    std::normal_distribution<double> nd(0.0, 1.0);
    double worst = 0;
    for (int trial = 0; trial < 20; ++trial) {
        double M[NC], xi[NL];
        for (auto &v : M) v = nd(rng);
        for (auto &v : xi) v = nd(rng);
        double Ba[NL], dMa[NC], Va;
        LA::template contract<double, true>(M, (const double *)xi, (double *)Ba, dMa, Va);
        double G[NG], dg[NG], Bb[NL], dMb[NC] = {}, Vb;
        graphs<0>(M, G);
        LB::template trie<double, true>((const double *)G, (const double *)xi, (double *)Bb, (double *)dg, Vb);
        reverse<0>(M, dg, dMb);
        double sc = std::fabs(Va), e = std::fabs(Va - Vb);
        for (int k = 0; k < NL; ++k) { sc = std::fmax(sc, std::fabs(Ba[k])); e = std::fmax(e, std::fabs(Ba[k] - Bb[k])); }
        double sd = 0, ed = 0;
        for (int k = 0; k < NC; ++k) { sd = std::fmax(sd, std::fabs(dMa[k])); ed = std::fmax(ed, std::fabs(dMa[k] - dMb[k])); }
        worst = std::fmax(worst, std::fmax(e / sc, ed / sd));
    }
    std::printf("level %d: worst relative difference %.3g\n", LV, worst);
    return worst < 1e-12 ? 0 : 1;
}
