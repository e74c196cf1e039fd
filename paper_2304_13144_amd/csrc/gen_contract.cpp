// Build-time generator: writes one HIP header per MTP level with the
// straight-line contraction program of that level.
//
// For a neighborhood with moment components M (see basis.hpp) the program
// computes
//   * every connected graph value g_G as a polynomial in M (sum over all edge
//     labelings of the product of tensor entries, Sec. II.A);
//   * the basis values B_alpha = prod g over the factors (eq. 6) and the site
//     energy V = sum_alpha xi_alpha B_alpha (eq. 2) by a nested (Horner-like)
//     walk over the trie of factor sequences: every prefix of a basis
//     function is itself a basis function, so trie nodes are basis functions;
//   * dV/dg_G along the same walk and dV/dM_k by reverse accumulation through
//     each graph polynomial.
//
// usage: gen_contract <out_dir> <level>...
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <functional>
#include <iostream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "basis.hpp"

using namespace mtp;

namespace {

struct Counter {
    long mul = 0, fma = 0, add = 0;
    long flops() const { return mul + add + 2 * fma; }
};

std::string lit(long c) { return "T(" + std::to_string(c) + ")"; }

struct Emitter {
    const Basis &B;
    std::ostringstream os;
    Counter fwd, rev;
    explicit Emitter(const Basis &b) : B(b) {}

    // Prefix products of the monomials of one graph, memoised: returns the
    // list of prefix nodes in creation order (each = parent * M[k]).
    struct PNode {
        int parent;     // -1: the node is M[k] itself
        int k;
        std::string name;
    };

    std::vector<PNode> prefixes(const std::vector<Monomial> &poly, std::vector<int> &term_node,
                                const std::string &tag) {
        std::vector<PNode> nodes;
        std::map<std::vector<int>, int> memo;
        for (auto &t : poly) {
            std::vector<int> pre;
            int cur = -1;
            for (int k : t.comp) {
                pre.push_back(k);
                auto it = memo.find(pre);
                if (it != memo.end()) {
                    cur = it->second;
                    continue;
                }
                PNode nd;
                nd.parent = cur;
                nd.k = k;
                nd.name = cur < 0 ? ("M[" + std::to_string(k) + "]") : (tag + std::to_string(nodes.size()));
                memo[pre] = (int)nodes.size();
                cur = (int)nodes.size();
                nodes.push_back(nd);
            }
            term_node.push_back(cur);
        }
        return nodes;
    }

    void emit_products(const std::vector<PNode> &nodes, Counter &c, const char *ind) {
        for (auto &nd : nodes)
            if (nd.parent >= 0) {
                os << ind << "const T " << nd.name << " = " << nodes[nd.parent].name << " * M[" << nd.k << "];\n";
                c.mul++;
            }
    }

    // Graph values of the graphs in `gl`.  to_array: written to gout[G] instead
    // of local variables g<G>.
    void graphs_forward(const std::vector<int> &gl, bool to_array) {
        os << "  // graph values\n";
        for (int G : gl) {
            auto &poly = B.polys[G];
            const std::string gv = to_array ? "acc" : "g" + std::to_string(G);
            if (!to_array) os << "  T " << gv << ";";
            os << "  // " << B.graphs[G].str() << ", " << poly.size() << " monomials\n";
            os << "  {\n";
            if (to_array) os << "    T acc;\n";
            std::vector<int> tn;
            auto nodes = prefixes(poly, tn, "p");
            emit_products(nodes, fwd, "    ");
            for (size_t t = 0; t < poly.size(); ++t) {
                const std::string &v = nodes[tn[t]].name;
                const long c = poly[t].coef;
                if (t == 0) {
                    if (c == 1) os << "    " << gv << " = " << v << ";\n";
                    else { os << "    " << gv << " = " << lit(c) << " * " << v << ";\n"; fwd.mul++; }
                } else {
                    if (c == 1) { os << "    " << gv << " += " << v << ";\n"; fwd.add++; }
                    else { os << "    " << gv << " = fma(" << lit(c) << ", " << v << ", " << gv << ");\n"; fwd.fma++; }
                }
            }
            if (to_array) os << "    gout[" << G << "] = acc;\n";
            os << "  }\n";
        }
    }

    // trie over sorted factor sequences
    struct TNode {
        int alpha = -1;
        std::map<int, int> child;   // graph id -> node
    };
    std::vector<TNode> trie;

    void build_trie() {
        trie.assign(1, TNode{});
        for (int a = 0; a < B.n_lin(); ++a) {
            int cur = 0;
            for (int g : B.funcs[a]) {
                auto it = trie[cur].child.find(g);
                if (it == trie[cur].child.end()) {
                    trie.push_back(TNode{});
                    trie[cur].child[g] = (int)trie.size() - 1;
                    cur = (int)trie.size() - 1;
                } else {
                    cur = it->second;
                }
            }
            trie[cur].alpha = a;
        }
        for (size_t n = 1; n < trie.size(); ++n)
            if (trie[n].alpha < 0) throw std::runtime_error("trie node without basis function");
    }

    std::vector<bool> dg_set;

    void visit(int node, int depth, const std::string &ind) {
        for (auto &kv : trie[node].child) {
            const int G = kv.first, c = kv.second;
            const std::string bd = "b" + std::to_string(depth), bd1 = "b" + std::to_string(depth + 1);
            const std::string wd = "w" + std::to_string(depth), wd1 = "w" + std::to_string(depth + 1);
            const std::string g = "g" + std::to_string(G), dg = "dg" + std::to_string(G);
            os << ind << "{\n";
            const std::string in2 = ind + "  ";
            if (depth == 0) os << in2 << "const T " << bd1 << " = " << g << ";\n";
            else { os << in2 << "const T " << bd1 << " = " << bd << " * " << g << ";\n"; trie_count.mul++; }
            os << in2 << "if (WB) Bout[" << trie[c].alpha << "] = " << bd1 << ";\n";
            os << in2 << "T " << wd1 << " = xi[" << trie[c].alpha << "];\n";
            visit(c, depth + 1, in2);
            // dV/dg_G gets B(parent) * W(child); W(parent) += g_G * W(child)
            if (depth == 0) {
                if (!dg_set[G]) { os << in2 << dg << " = " << wd1 << ";\n"; dg_set[G] = true; }
                else { os << in2 << dg << " += " << wd1 << ";\n"; trie_count.add++; }
            } else {
                if (!dg_set[G]) { os << in2 << dg << " = " << bd << " * " << wd1 << ";\n"; dg_set[G] = true; trie_count.mul++; }
                else { os << in2 << dg << " = fma(" << bd << ", " << wd1 << ", " << dg << ");\n"; trie_count.fma++; }
            }
            os << in2 << wd << " = fma(" << g << ", " << wd1 << ", " << wd << ");\n";
            trie_count.fma++;
            os << ind << "}\n";
        }
    }
    Counter trie_count;

    void trie_walk(bool arrays) {
        build_trie();
        os << "  // basis values, site energy and dV/dg by a walk over the factor trie\n";
        if (arrays)
            for (size_t G = 0; G < B.graphs.size(); ++G) os << "  const T g" << G << " = gin[" << G << "];\n";
        for (size_t G = 0; G < B.graphs.size(); ++G) os << "  T dg" << G << ";\n";
        dg_set.assign(B.graphs.size(), false);
        trie_count = Counter{};
        os << "  T w0 = T(0);\n";
        visit(0, 0, "  ");
        os << "  V = w0;\n";
        for (size_t G = 0; G < B.graphs.size(); ++G)
            if (!dg_set[G]) os << "  dg" << G << " = T(0);\n";
        if (arrays)
            for (size_t G = 0; G < B.graphs.size(); ++G) os << "  dgout[" << G << "] = dg" << G << ";\n";
    }

    void graphs_reverse(const std::vector<int> &gl, bool dg_array) {
        os << "  // dV/dM by reverse accumulation through the graph polynomials\n";
        std::vector<bool> dm_set(B.n_comp(), false);
        for (int G : gl) {
            auto &poly = B.polys[G];
            os << "  {\n";
            if (dg_array) os << "    const T dg" << G << " = dgin[" << G << "];\n";
            std::vector<int> tn;
            auto nodes = prefixes(poly, tn, "q");
            emit_products(nodes, rev, "    ");
            // adjoints of prefix nodes
            std::vector<std::string> adj(nodes.size());
            std::vector<bool> aset(nodes.size(), false);
            for (size_t n = 0; n < nodes.size(); ++n) adj[n] = "a" + std::to_string(n);
            auto add_adj = [&](int n, const std::string &expr_mul_a, const std::string &expr_mul_b, bool is_mul) {
                // adj[n] += a * b (is_mul) or adj[n] += a (expr_mul_b empty)
                if (!aset[n]) {
                    os << "    T " << adj[n] << " = " << expr_mul_a;
                    if (is_mul) { os << " * " << expr_mul_b; rev.mul++; }
                    os << ";\n";
                    aset[n] = true;
                } else if (is_mul) {
                    os << "    " << adj[n] << " = fma(" << expr_mul_a << ", " << expr_mul_b << ", " << adj[n] << ");\n";
                    rev.fma++;
                } else {
                    os << "    " << adj[n] << " += " << expr_mul_a << ";\n";
                    rev.add++;
                }
            };
            const std::string dg = "dg" + std::to_string(G);
            for (size_t t = 0; t < poly.size(); ++t) {
                const long c = poly[t].coef;
                if (c == 1) add_adj(tn[t], dg, "", false);
                else add_adj(tn[t], lit(c), dg, true);
            }
            auto add_dm = [&](int k, const std::string &a, const std::string &b) {
                if (!dm_set[k]) {
                    os << "    dM[" << k << "] = " << a;
                    if (!b.empty()) { os << " * " << b; rev.mul++; }
                    os << ";\n";
                    dm_set[k] = true;
                } else if (!b.empty()) {
                    os << "    dM[" << k << "] = fma(" << a << ", " << b << ", dM[" << k << "]);\n";
                    rev.fma++;
                } else {
                    os << "    dM[" << k << "] += " << a << ";\n";
                    rev.add++;
                }
            };
            for (int n = (int)nodes.size() - 1; n >= 0; --n) {
                if (!aset[n]) continue;
                const auto &nd = nodes[n];
                if (nd.parent < 0) {
                    add_dm(nd.k, adj[n], "");
                } else {
                    add_adj(nd.parent, adj[n], "M[" + std::to_string(nd.k) + "]", true);
                    add_dm(nd.k, adj[n], nodes[nd.parent].name);
                }
            }
            os << "  }\n";
        }
        for (int k = 0; k < B.n_comp(); ++k)
            if (!dm_set[k]) os << "  dM[" << k << "] = T(0);\n";
    }
};

void write_level(const std::string &dir, int level) {
    Basis B = build_basis(level);
    Emitter em(B);
    std::vector<int> all(B.graphs.size());
    for (size_t G = 0; G < all.size(); ++G) all[G] = (int)G;
    em.graphs_forward(all, false);
    std::string fwd = em.os.str();
    em.os.str("");
    em.trie_walk(false);
    std::string walk = em.os.str();
    em.os.str("");
    em.graphs_reverse(all, false);
    std::string rev = em.os.str();
    const Counter cf = em.fwd, ct = em.trie_count, cr = em.rev;

    // Split of the graphs over np wavefronts (largest first onto the least
    // loaded part; cost = monomial terms x degree): the four-part program of
    // the four-wavefront kernels and the eight-part one of the eight-wavefront
    // kernel.
    struct Split {
        std::vector<int> part;
        std::vector<std::string> pf, pr;
    };
    auto split = [&](int np) {
        Split sp;
        sp.part.assign(B.graphs.size(), 0);
        std::vector<std::pair<long, int>> cost;
        for (size_t G = 0; G < B.graphs.size(); ++G) {
            long c = 0;
            for (auto &t : B.polys[G]) c += (long)t.comp.size();
            cost.push_back({c, (int)G});
        }
        std::sort(cost.begin(), cost.end(), [](auto &a, auto &b) { return a.first > b.first || (a.first == b.first && a.second < b.second); });
        std::vector<long> load(np, 0);
        for (auto &c : cost) {
            int best = 0;
            for (int q = 1; q < np; ++q)
                if (load[q] < load[best]) best = q;
            sp.part[c.second] = best;
            load[best] += c.first;
        }
        sp.pf.resize(np);
        sp.pr.resize(np);
        for (int q = 0; q < np; ++q) {
            std::vector<int> gl;
            for (size_t G = 0; G < B.graphs.size(); ++G)
                if (sp.part[G] == q) gl.push_back((int)G);
            em.os.str("");
            em.graphs_forward(gl, true);
            sp.pf[q] = em.os.str();
            em.os.str("");
            em.graphs_reverse(gl, true);
            sp.pr[q] = em.os.str();
        }
        return sp;
    };
    const int NPART = 4, NPART8 = 8;
    const Split s4 = split(NPART), s8 = split(NPART8);
    em.os.str("");
    em.trie_walk(true);
    std::string walk_arrays = em.os.str();

    const int NC = B.n_comp();
    std::ostringstream h;
    h << "// generated by gen_contract for MTP level " << level << "; do not edit.\n";
    h << "// " << B.graphs.size() << " connected graphs, " << B.n_lin() << " basis functions, "
      << NC << " moment components, " << B.n_rad << " radial functions.\n";
    h << "#pragma once\n\n";
    h << "template <> struct Level<" << level << "> {\n";
    h << "  static constexpr int NC = " << NC << ";\n";
    h << "  static constexpr int NLIN = " << B.n_lin() << ";\n";
    h << "  static constexpr int NRAD = " << B.n_rad << ";\n";
    h << "  static constexpr int NGRAPH = " << B.graphs.size() << ";\n";
    int maxnu = 0;
    for (auto &c : B.comps) maxnu = std::max(maxnu, c.nu);
    h << "  static constexpr int MAXNU = " << maxnu << ";\n";
    h << "  // flops of the contraction program per neighborhood (mul/add = 1, fma = 2)\n";
    h << "  static constexpr long FLOPS_GRAPHS = " << cf.flops() << ";\n";
    h << "  static constexpr long FLOPS_TRIE = " << ct.flops() << ";\n";
    h << "  static constexpr long FLOPS_REVERSE = " << cr.flops() << ";\n";
    h << "  static constexpr int NPART = " << NPART << ";\n";
    h << "  static constexpr int graph_part[" << B.graphs.size() << "] = {";
    for (size_t G = 0; G < B.graphs.size(); ++G) h << (G ? "," : "") << s4.part[G];
    h << "};\n";
    h << "  static constexpr int NPART8 = " << NPART8 << ";\n";
    h << "  static constexpr int graph_part8[" << B.graphs.size() << "] = {";
    for (size_t G = 0; G < B.graphs.size(); ++G) h << (G ? "," : "") << s8.part[G];
    h << "};\n";
    auto arr = [&](const char *name, auto f) {
        h << "  static constexpr int " << name << "[" << NC << "] = {";
        for (int k = 0; k < NC; ++k) h << (k ? "," : "") << f(B.comps[k]);
        h << "};\n";
    };
    arr("comp_mu", [](const Component &c) { return c.mu; });
    arr("comp_nu", [](const Component &c) { return c.nu; });
    arr("comp_mono", [](const Component &c) { return monomial_index(c.e[0], c.e[1], c.e[2]); });
    for (int ax = 0; ax < 3; ++ax) {
        std::string nm = std::string("comp_dmono") + "xyz"[ax];
        arr(nm.c_str(), [ax](const Component &c) {
            if (c.e[ax] == 0) return -1;
            int e[3] = {c.e[0], c.e[1], c.e[2]};
            e[ax]--;
            return monomial_index(e[0], e[1], e[2]);
        });
        std::string nf = std::string("comp_dfac") + "xyz"[ax];
        arr(nf.c_str(), [ax](const Component &c) { return c.e[ax]; });
    }
    // T: value type (double, float, or a dual number for tangents); XP: anything
    // indexable giving xi_alpha; BP: anything indexable receiving B_alpha.
    h << "\n  template <typename T, bool WB, typename XP, typename BP>\n";
    h << "  __device__ __forceinline__ static void contract(const T (&M)[NC], XP xi, BP Bout, T (&dM)[NC], T &V) {\n";
    h << fwd << walk << rev;
    h << "  }\n";
    // the same program in parts: graph values of part P, the trie walk from
    // all graph values, and the reverse pass of part P (dM zero elsewhere)
    auto parts = [&](const char *name, const char *sig, const std::vector<std::string> &body) {
        h << "\n  template <int P, typename T, typename MP>\n";
        h << "  __device__ __forceinline__ static void " << name << sig << " {\n";
        for (size_t q = 0; q < body.size(); ++q)
            h << "  " << (q ? "else " : "") << "if constexpr (P == " << q << ") {\n" << body[q] << "  }\n";
        h << "  }\n";
    };
    parts("graphs_part", "(MP M, T *gout)", s4.pf);
    parts("graphs_part8", "(MP M, T *gout)", s8.pf);
    h << "\n  template <typename T, bool WB, typename XP, typename BP>\n";
    h << "  __device__ __forceinline__ static void trie(const T *gin, XP xi, BP Bout, T *dgout, T &V) {\n";
    h << walk_arrays << "  }\n";
    parts("reverse_part", "(MP M, const T *dgin, T (&dM)[NC])", s4.pr);
    parts("reverse_part8", "(MP M, const T *dgin, T (&dM)[NC])", s8.pr);
    h << "};\n";
    std::ofstream out(dir + "/mtp_level" + std::to_string(level) + ".inc");
    out << h.str();
    std::cout << "level " << level << ": graphs " << B.graphs.size() << " basis " << B.n_lin() << " comps " << NC
              << " flops graphs " << cf.flops() << " trie " << ct.flops() << " reverse " << cr.flops() << "\n";
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 3) {
        std::cerr << "usage: gen_contract <out_dir> <level>...\n";
        return 2;
    }
    for (int i = 2; i < argc; ++i) write_level(argv[1], std::atoi(argv[i]));
    return 0;
}
