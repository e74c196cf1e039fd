// Basis of the Moment Tensor Potential and its contraction program.
//
// The level of a moment is lev M_{mu,nu} = 2 + 4 mu + nu and the level of a
// product of moments is the sum of the factors' levels (MLIP-3 paper,
// Sec. II.A, eqs. 5-6); the basis holds every full contraction to a scalar
// whose level is at most lev_max.  Admitted contractions (the paper shows
// examples only): multigraphs over moments with nu <= 3, no contraction of a
// tensor with itself, at most two contracted index pairs between two
// tensors; a basis function is a product of connected contractions.  This
// reproduces N_lin = 5, N_rad = 2 at level 6 and |theta| = 26 / 54 / 125 at
// levels 8 / 12 / 16 for one species (Sec. II.A, Sec. IV).
//
// Order of the basis (fixes the column order of xi): a connected graph's
// nodes are sorted by (mu, nu) and, among node orders keeping that sort, the
// lexicographically smallest upper-triangle edge-multiplicity vector is
// canonical; graphs are ordered by (level, #nodes, labels, edges); a basis
// function lists its factors in graph order and functions are ordered by
// (level, #factors, factor sequence).
//
// Moments are stored by symmetric components: M_{mu,nu} has one component
// per multiset {i_1..i_nu} of Cartesian indices, i.e. per exponent triple
// (a, b, c), a + b + c = nu, with value sum_j f_mu(r_j) x^a y^b z^c.
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace mtp {

struct Label {
    int mu, nu;
    bool operator<(const Label &o) const { return mu != o.mu ? mu < o.mu : nu < o.nu; }
    bool operator==(const Label &o) const { return mu == o.mu && nu == o.nu; }
    bool operator!=(const Label &o) const { return !(*this == o); }
};

inline int moment_level(int mu, int nu) { return 2 + 4 * mu + nu; }

struct CGraph {                      // connected contraction graph
    std::vector<Label> labels;       // sorted
    std::vector<int> edges;          // e_pq, p < q, row-major, canonical
    int level() const;
    int n() const { return (int)labels.size(); }
    std::string str() const;
};

// One monomial of a graph polynomial: coef * prod M[comp[i]].
struct Monomial {
    long coef;
    std::vector<int> comp;           // sorted global component ids
};

struct Component {
    int mu, nu;
    int e[3];                        // exponents of x, y, z
};

struct Basis {
    int level = 0;
    std::vector<CGraph> graphs;                      // sorted connected graphs
    std::vector<std::vector<int>> funcs;             // basis functions: graph ids, sorted
    std::vector<Label> moments;                      // moments used, sorted
    std::vector<Component> comps;                    // symmetric components, grouped by moment
    std::vector<std::vector<Monomial>> polys;        // per graph
    int n_rad = 0;

    int n_lin() const { return (int)funcs.size(); }
    int n_comp() const { return (int)comps.size(); }
    std::string describe() const;                    // one basis function per line
};

// Enumerates the basis of a level (0 < level <= 40).
Basis build_basis(int level);

// Index of the monomial x^a y^b z^c in the list of all monomials of degree
// <= 3 ordered by degree, then lexicographically by the sorted index tuple
// (1; x y z; xx xy xz yy yz zz; xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz).
int monomial_index(int a, int b, int c);

}  // namespace mtp
