// Basis enumeration and graph polynomials (see basis.hpp for the rule).
#include "basis.hpp"

#include <algorithm>
#include <functional>
#include <set>
#include <sstream>
#include <stdexcept>
#include <tuple>

namespace mtp {

int CGraph::level() const {
    int s = 0;
    for (auto &l : labels) s += moment_level(l.mu, l.nu);
    return s;
}

std::string CGraph::str() const {
    std::ostringstream os;
    os << "[";
    for (int p = 0; p < n(); ++p) os << (p ? " " : "") << "M" << labels[p].mu << labels[p].nu;
    os << "]";
    std::string e;
    int k = 0;
    for (int p = 0; p < n(); ++p)
        for (int q = p + 1; q < n(); ++q, ++k)
            if (edges[k]) {
                if (!e.empty()) e += ",";
                e += std::to_string(p) + "-" + std::to_string(q) + ":" + std::to_string(edges[k]);
            }
    if (!e.empty()) os << "(" << e << ")";
    return os.str();
}

int monomial_index(int a, int b, int c) {
    // degree d block starts at (d)(d+1)(d+2)/6; inside a block the sorted
    // index tuples (0...0 1...1 2...2) are in lexicographic order, which is
    // decreasing a, then decreasing b.
    const int d = a + b + c;
    int idx = d * (d + 1) * (d + 2) / 6;
    for (int aa = d; aa > a; --aa) idx += d - aa + 1;   // tuples with more x's
    idx += (d - a) - b;                                  // then more y's first
    return idx;
}

namespace {

using EdgeMat = std::vector<std::vector<int>>;

bool is_connected(int n, const EdgeMat &m) {
    std::vector<int> seen(n, 0), stack{0};
    seen[0] = 1;
    int count = 1;
    while (!stack.empty()) {
        int p = stack.back();
        stack.pop_back();
        for (int q = 0; q < n; ++q)
            if (m[p][q] && !seen[q]) {
                seen[q] = 1;
                ++count;
                stack.push_back(q);
            }
    }
    return count == n;
}

// Smallest upper-triangle vector over permutations that only exchange nodes
// with equal labels (labels are sorted, so such nodes are contiguous).
std::vector<int> canonical_edges(const std::vector<Label> &lab, const EdgeMat &m) {
    const int n = (int)lab.size();
    std::vector<int> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    std::vector<std::pair<int, int>> groups;  // [begin, end)
    for (int i = 0; i < n;) {
        int j = i;
        while (j < n && lab[j] == lab[i]) ++j;
        groups.push_back({i, j});
        i = j;
    }
    std::vector<int> best;
    std::function<void(size_t)> rec = [&](size_t g) {
        if (g == groups.size()) {
            std::vector<int> v;
            for (int p = 0; p < n; ++p)
                for (int q = p + 1; q < n; ++q) v.push_back(m[perm[p]][perm[q]]);
            if (best.empty() || v < best) best = v;
            return;
        }
        auto b = perm.begin() + groups[g].first, e = perm.begin() + groups[g].second;
        std::sort(b, e);
        do {
            rec(g + 1);
        } while (std::next_permutation(b, e));
    };
    rec(0);
    return best;
}

using GKey = std::tuple<int, int, std::vector<Label>, std::vector<int>>;

GKey graph_key(const CGraph &g) { return GKey(g.level(), g.n(), g.labels, g.edges); }

}  // namespace

Basis build_basis(int level) {
    if (level < 2 || level > 40) throw std::invalid_argument("level out of range");
    Basis B;
    B.level = level;

    // candidate node labels
    std::vector<Label> scalars, tensors;
    for (int mu = 0; moment_level(mu, 0) <= level; ++mu)
        for (int nu = 0; nu <= 3; ++nu)
            if (moment_level(mu, nu) <= level) (nu ? tensors : scalars).push_back({mu, nu});
    std::sort(tensors.begin(), tensors.end());

    std::set<GKey> found;
    for (auto &s : scalars) found.insert(GKey(moment_level(s.mu, s.nu), 1, std::vector<Label>{s}, std::vector<int>{}));

    // multisets of tensor labels (non-decreasing index sequences) within budget
    std::vector<Label> cur;
    std::function<void(size_t, int)> grow = [&](size_t from, int budget) {
        if (cur.size() >= 2) {
            const int n = (int)cur.size();
            EdgeMat m(n, std::vector<int>(n, 0));
            std::vector<int> rem(n);
            for (int p = 0; p < n; ++p) rem[p] = cur[p].nu;
            // assign multiplicities pair by pair
            std::vector<std::pair<int, int>> pairs;
            for (int p = 0; p < n; ++p)
                for (int q = p + 1; q < n; ++q) pairs.push_back({p, q});
            std::function<void(size_t)> assign = [&](size_t k) {
                if (k == pairs.size()) {
                    for (int p = 0; p < n; ++p)
                        if (rem[p]) return;
                    if (!is_connected(n, m)) return;
                    int lev = 0;
                    for (auto &l : cur) lev += moment_level(l.mu, l.nu);
                    found.insert(GKey(lev, n, cur, canonical_edges(cur, m)));
                    return;
                }
                const int p = pairs[k].first, q = pairs[k].second;
                // node p gets no further pairs after its last one: prune
                const int top = std::min({2, rem[p], rem[q]});
                for (int e = 0; e <= top; ++e) {
                    rem[p] -= e;
                    rem[q] -= e;
                    m[p][q] = m[q][p] = e;
                    bool ok = true;
                    if (q == n - 1 && rem[p] != 0) ok = false;   // p's row is complete
                    if (ok) assign(k + 1);
                    rem[p] += e;
                    rem[q] += e;
                    m[p][q] = m[q][p] = 0;
                }
            };
            assign(0);
        }
        for (size_t t = from; t < tensors.size(); ++t) {
            const int lv = moment_level(tensors[t].mu, tensors[t].nu);
            if (lv > budget) continue;
            cur.push_back(tensors[t]);
            grow(t, budget - lv);
            cur.pop_back();
        }
    };
    grow(0, level);

    for (auto &k : found) {
        CGraph g;
        g.labels = std::get<2>(k);
        g.edges = std::get<3>(k);
        B.graphs.push_back(g);
    }
    // std::set already orders by the key tuple (level, n, labels, edges)

    // basis functions: multisets of graph ids within the level budget
    std::vector<int> fcur;
    std::function<void(int, int)> pick = [&](int from, int budget) {
        if (!fcur.empty()) B.funcs.push_back(fcur);
        for (int g = from; g < (int)B.graphs.size(); ++g) {
            const int lv = B.graphs[g].level();
            if (lv > budget) continue;
            fcur.push_back(g);
            pick(g, budget - lv);
            fcur.pop_back();
        }
    };
    pick(0, level);
    auto flevel = [&](const std::vector<int> &f) {
        int s = 0;
        for (int g : f) s += B.graphs[g].level();
        return s;
    };
    std::sort(B.funcs.begin(), B.funcs.end(), [&](const std::vector<int> &a, const std::vector<int> &b) {
        const int la = flevel(a), lb = flevel(b);
        if (la != lb) return la < lb;
        if (a.size() != b.size()) return a.size() < b.size();
        return a < b;   // graph ids follow the graph order
    });

    // moments used and their symmetric components
    std::set<Label> used;
    for (auto &f : B.funcs)
        for (int g : f)
            for (auto &l : B.graphs[g].labels) used.insert(l);
    B.moments.assign(used.begin(), used.end());
    std::map<std::tuple<int, int, int, int, int>, int> comp_id;   // (mu, nu, a, b, c)
    for (auto &l : B.moments) {
        B.n_rad = std::max(B.n_rad, l.mu + 1);
        // sorted index tuples in lexicographic order = decreasing a, then b
        for (int a = l.nu; a >= 0; --a)
            for (int b = l.nu - a; b >= 0; --b) {
                Component c{l.mu, l.nu, {a, b, l.nu - a - b}};
                comp_id[{l.mu, l.nu, a, b, l.nu - a - b}] = (int)B.comps.size();
                B.comps.push_back(c);
            }
    }

    // graph polynomials over the components: sum over all 3^E labelings
    for (auto &g : B.graphs) {
        const int n = g.n();
        std::vector<std::pair<int, int>> slots;   // edge slots (p, q)
        int k = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q, ++k)
                for (int e = 0; e < g.edges[k]; ++e) slots.push_back({p, q});
        const int E = (int)slots.size();
        long total = 1;
        for (int e = 0; e < E; ++e) total *= 3;
        std::map<std::vector<int>, long> acc;
        std::vector<int> ax(E);
        for (long code = 0; code < total; ++code) {
            long c = code;
            for (int e = 0; e < E; ++e) {
                ax[e] = (int)(c % 3);
                c /= 3;
            }
            std::vector<std::array<int, 3>> cnt(n, {0, 0, 0});
            for (int e = 0; e < E; ++e) {
                cnt[slots[e].first][ax[e]]++;
                cnt[slots[e].second][ax[e]]++;
            }
            std::vector<int> mono;
            for (int p = 0; p < n; ++p)
                mono.push_back(comp_id.at({g.labels[p].mu, g.labels[p].nu, cnt[p][0], cnt[p][1], cnt[p][2]}));
            std::sort(mono.begin(), mono.end());
            acc[mono] += 1;
        }
        std::vector<Monomial> poly;
        for (auto &kv : acc) poly.push_back({kv.second, kv.first});
        B.polys.push_back(poly);
    }
    return B;
}

std::string Basis::describe() const {
    std::ostringstream os;
    for (auto &f : funcs) {
        for (size_t i = 0; i < f.size(); ++i) os << (i ? "*" : "") << graphs[f[i]].str();
        os << "\n";
    }
    return os.str();
}

}  // namespace mtp
