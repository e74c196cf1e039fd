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
#include <set>
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
    bool stream = false;   // graph values read from gin[] at each use, dV/dg accumulated in dgout[]

    void visit(int node, int depth, const std::string &ind) {
        for (auto &kv : trie[node].child) {
            const int G = kv.first, c = kv.second;
            const std::string bd = "b" + std::to_string(depth), bd1 = "b" + std::to_string(depth + 1);
            const std::string wd = "w" + std::to_string(depth), wd1 = "w" + std::to_string(depth + 1);
            const std::string g = stream ? "gin[" + std::to_string(G) + "]" : "g" + std::to_string(G);
            const std::string dg = stream ? "dgout[" + std::to_string(G) + "]" : "dg" + std::to_string(G);
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
            // streamed walk: after each node of the first two depths, dV/dg
            // goes back to memory; after every node the parent's sum is
            // formed here, not deferred to its use
            if (stream) os << ind << (depth <= 1 ? "MTP_STAGE_SYNC(" : "MTP_STAGE_KEEP(") << wd << ");\n";
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

    // Horner form of one graph polynomial over the tree of its monomials'
    // factor prefixes: S(n) = coef(n) + sum over children c of M[k_c] S(c), so
    // that g = S(root) and, with q(n) = dV/dg x the product of the factors
    // on the path to n, dV/dM[k_c] gets q(parent c) S(c) at every node c.  The
    // walk is depth first: only one S and one q per depth are live (the
    // prefix-product form holds every prefix of the graph at once).
    struct HTree {
        std::vector<int> k;
        std::vector<long> coef;
        std::vector<std::vector<int>> ch;
        std::vector<int> roots;
    };
    static HTree htree(const std::vector<Monomial> &poly) {
        HTree t;
        std::map<std::vector<int>, int> memo;
        for (auto &m : poly) {
            std::vector<int> pre;
            int cur = -1;
            for (int k : m.comp) {
                pre.push_back(k);
                auto it = memo.find(pre);
                if (it != memo.end()) {
                    cur = it->second;
                    continue;
                }
                const int n = (int)t.k.size();
                t.k.push_back(k);
                t.coef.push_back(0);
                t.ch.emplace_back();
                (cur < 0 ? t.roots : t.ch[cur]).push_back(n);
                memo[pre] = n;
                cur = n;
            }
            t.coef[cur] += m.coef;
        }
        return t;
    }
    std::vector<bool> hdm_set;
    void h_dm(int k, const std::string &a, long c, Counter &cnt) {   // dM[k] += a (c = 1) or a * c
        const std::string term = c == 1 ? a : lit(c) + " * " + a;
        if (!hdm_set[k]) {
            os << "dM[" << k << "] = " << term << ";\n";
            if (c != 1) cnt.mul++;
            hdm_set[k] = true;
        } else if (c == 1) {
            os << "dM[" << k << "] += " << a << ";\n";
            cnt.add++;
        } else {
            os << "dM[" << k << "] = fma(" << lit(c) << ", " << a << ", dM[" << k << "]);\n";
            cnt.fma++;
        }
    }
    // emits the accumulation of the children `kids` of a node into a<d> (and
    // with rev the dV/dM terms, q: the name of q(node))
    void h_children(const HTree &t, const std::vector<int> &kids, int d, bool rev, const std::string &q, Counter &cnt) {
        const std::string ad = "a" + std::to_string(d);
        for (int c : kids) {
            const std::string Mk = "M[" + std::to_string(t.k[c]) + "]";
            if (t.ch[c].empty()) {   // leaf: S(c) = coef(c)
                const long cf = t.coef[c];
                if (cf == 1) { os << ad << " += " << Mk << ";\n"; cnt.add++; }
                else { os << ad << " = fma(" << lit(cf) << ", " << Mk << ", " << ad << ");\n"; cnt.fma++; }
                if (rev) h_dm(t.k[c], q, cf, cnt);
                continue;
            }
            const std::string a1 = "a" + std::to_string(d + 1), q1 = "q" + std::to_string(d + 1);
            os << "{\n";
            if (rev) { os << "const T " << q1 << " = " << q << " * " << Mk << ";\n"; cnt.mul++; }
            os << "T " << a1 << " = " << (t.coef[c] ? lit(t.coef[c]) : std::string("T(0)")) << ";\n";
            h_children(t, t.ch[c], d + 1, rev, q1, cnt);
            if (rev) h_dm(t.k[c], q + " * " + a1, 1, cnt), cnt.mul++;
            os << ad << " = fma(" << Mk << ", " << a1 << ", " << ad << ");\n";
            cnt.fma++;
            os << "}\nMTP_STAGE_KEEP(" << ad << ");\n";
        }
    }
    // graph values of `gl` in Horner form, written to gout[G]
    void graphs_forward_horner(const std::vector<int> &gl) {
        os << "  // graph values (Horner form over the factor-prefix tree)\n";
        for (int G : gl) {
            const HTree t = htree(B.polys[G]);
            os << "  {  // " << B.graphs[G].str() << ", " << B.polys[G].size() << " monomials\n";
            os << "T a0 = T(0);\n";
            h_children(t, t.roots, 0, false, "", fwd);
            os << "gout[" << G << "] = a0;\n  }\n  MTP_STAGE_SCHED();\n";
        }
    }
    // dV/dM of the graphs `gl` in Horner form (dg from dgin[G])
    void graphs_reverse_horner(const std::vector<int> &gl) {
        os << "  // dV/dM by reverse accumulation (Horner form over the factor-prefix tree)\n";
        hdm_set.assign(B.n_comp(), false);
        for (int G : gl) {
            const HTree t = htree(B.polys[G]);
            os << "  {  // " << B.graphs[G].str() << "\n";
            os << "const T q0 = dgin[" << G << "];\nT a0 = T(0);\n";
            h_children(t, t.roots, 0, true, "q0", rev);
            os << "(void)a0;\n  }\n  MTP_STAGE_SCHED();\n";
        }
        for (int k = 0; k < B.n_comp(); ++k)
            if (!hdm_set[k]) os << "  dM[" << k << "] = T(0);\n";
    }

    // The trie walk with every graph value read where it is used and dV/dg
    // accumulated in place (gin, dgout: accessors into memory), so that the
    // 2 x NGRAPH values are not all held in registers.
    void trie_walk_stream() {
        build_trie();
        os << "  // basis values, site energy and dV/dg by a walk over the factor trie\n";
        dg_set.assign(B.graphs.size(), false);
        trie_count = Counter{};
        stream = true;
        os << "  T w0 = T(0);\n";
        visit(0, 0, "  ");
        stream = false;
        os << "  V = w0;\n";
        for (size_t G = 0; G < B.graphs.size(); ++G)
            if (!dg_set[G]) os << "  dgout[" << G << "] = T(0);\n";
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

// Levels with more connected graphs than this get the staged program: graph
// values, trie walk and reverse pass as separate kernels (graph values and
// dV/dg pass through memory), each split into parts that compile apart.
constexpr int STAGED_GRAPHS = 128;
constexpr int STAGE_G = 8, STAGE_R = 16;

// Split for the staged program: graphs (largest first) go to the part whose
// set of moment components grows least, among the parts whose cost stays
// within 15 % of the mean (else the least loaded part): a part then reads
// and writes few components (level 24: at most 44 of 91 in 8 parts, 38 in
// 16), which its kernel holds in registers.
std::vector<int> cluster_graphs(const Basis &B, int np) {
    const size_t ng = B.graphs.size();
    std::vector<std::set<int>> comp(ng);
    std::vector<long> cost(ng, 0);
    long total = 0;
    for (size_t G = 0; G < ng; ++G) {
        for (auto &t : B.polys[G]) {
            comp[G].insert(t.comp.begin(), t.comp.end());
            cost[G] += (long)t.comp.size();
        }
        total += cost[G];
    }
    const double cap = 1.15 * (double)total / np;
    std::vector<int> order(ng), part(ng, 0);
    for (size_t G = 0; G < ng; ++G) order[G] = (int)G;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<std::set<int>> uni(np);
    std::vector<long> load(np, 0);
    for (int G : order) {
        int best = -1;
        size_t bu = 0;
        for (int q = 0; q < np; ++q) {
            if (load[q] > 0 && load[q] + cost[G] > cap) continue;
            size_t u = uni[q].size();
            for (int k : comp[G]) u += uni[q].count(k) ? 0 : 1;
            if (best < 0 || u < bu || (u == bu && load[q] < load[best])) {
                best = q;
                bu = u;
            }
        }
        if (best < 0) best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        part[G] = best;
        uni[best].insert(comp[G].begin(), comp[G].end());
        load[best] += cost[G];
    }
    return part;
}

std::vector<int> part_components(const Basis &B, const std::vector<int> &gl) {
    std::set<int> u;
    for (int G : gl)
        for (auto &t : B.polys[G]) u.insert(t.comp.begin(), t.comp.end());
    return std::vector<int>(u.begin(), u.end());
}

void write_common(std::ostringstream &h, const Basis &B, int level) {
    const int NC = B.n_comp();
    h << "  static constexpr int NC = " << NC << ";\n";
    h << "  static constexpr int NLIN = " << B.n_lin() << ";\n";
    h << "  static constexpr int NRAD = " << B.n_rad << ";\n";
    h << "  static constexpr int NGRAPH = " << B.graphs.size() << ";\n";
    int maxnu = 0;
    for (auto &c : B.comps) maxnu = std::max(maxnu, c.nu);
    h << "  static constexpr int MAXNU = " << maxnu << ";\n";
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
}

// The staged program of a large level: mtp_level<L>.inc holds the constants
// and the trie walk; mtp_level<L>_g<P>.inc the graph values of part P
// (LevelGraphs<L, P>::run) and mtp_level<L>_r<P>.inc the reverse pass of part
// P (LevelReverse<L, P>::run), each included by its own translation unit.
void write_level_staged(const std::string &dir, int level, const Basis &B) {
    Emitter em(B);
    const std::vector<int> pg = cluster_graphs(B, STAGE_G), pr = cluster_graphs(B, STAGE_R);
    auto graphs_of = [&](const std::vector<int> &part, int q) {
        std::vector<int> gl;
        for (size_t G = 0; G < B.graphs.size(); ++G)
            if (part[G] == q) gl.push_back((int)G);
        return gl;
    };
    const std::string L = std::to_string(level);
    for (int q = 0; q < STAGE_G; ++q) {
        em.os.str("");
        em.graphs_forward_horner(graphs_of(pg, q));
        std::ofstream out(dir + "/mtp_level" + L + "_g" + std::to_string(q) + ".inc");
        out << "// generated by gen_contract for MTP level " << level << ", graph values of part " << q
            << "; do not edit.\n#pragma once\n\n";
        const std::vector<int> mc = part_components(B, graphs_of(pg, q));
        out << "template <> struct LevelGraphs<" << level << ", " << q << "> {\n";
        out << "  // the moment components this part reads\n";
        out << "  static constexpr int NM = " << mc.size() << ";\n  static constexpr int mcomp[" << std::max<size_t>(1, mc.size()) << "] = {";
        for (size_t i = 0; i < mc.size(); ++i) out << (i ? "," : "") << mc[i];
        if (mc.empty()) out << "0";
        out << "};\n";
        out << "  template <typename T, typename MP, typename GP>\n";
        out << "  __device__ __forceinline__ static void run(MP M, GP gout) {\n" << em.os.str() << "  }\n};\n";
    }
    for (int q = 0; q < STAGE_R; ++q) {
        em.os.str("");
        em.graphs_reverse_horner(graphs_of(pr, q));
        std::ofstream out(dir + "/mtp_level" + L + "_r" + std::to_string(q) + ".inc");
        out << "// generated by gen_contract for MTP level " << level << ", reverse pass of part " << q
            << "; do not edit.\n#pragma once\n\n";
        const std::vector<int> mc = part_components(B, graphs_of(pr, q));
        out << "template <> struct LevelReverse<" << level << ", " << q << "> {\n";
        out << "  // the moment components this part reads and whose dV/dM it adds to (the others stay zero)\n";
        out << "  static constexpr int NM = " << mc.size() << ";\n  static constexpr int mcomp[" << std::max<size_t>(1, mc.size()) << "] = {";
        for (size_t i = 0; i < mc.size(); ++i) out << (i ? "," : "") << mc[i];
        if (mc.empty()) out << "0";
        out << "};\n";
        out << "  template <typename T, typename MP, typename DP>\n";
        out << "  __device__ __forceinline__ static void run(MP M, DP dgin, T (&dM)[" << B.n_comp() << "]) {\n"
            << em.os.str() << "  }\n};\n";
    }
    em.os.str("");
    em.trie_walk_stream();
    const std::string walk = em.os.str();
    // flops of the whole program (the parts are disjoint)
    const Counter cf = em.fwd, cr = em.rev;   // every graph once in each (the parts are disjoint)
    std::ostringstream h;
    h << "// generated by gen_contract for MTP level " << level << "; do not edit.\n";
    h << "// " << B.graphs.size() << " connected graphs, " << B.n_lin() << " basis functions, " << B.n_comp()
      << " moment components, " << B.n_rad << " radial functions; staged program.\n";
    h << "#pragma once\n\n";
    h << "template <> struct Level<" << level << "> {\n";
    write_common(h, B, level);
    h << "  // flops of the contraction program per neighborhood (mul/add = 1, fma = 2)\n";
    h << "  static constexpr long FLOPS_GRAPHS = " << cf.flops() << ";\n";
    h << "  static constexpr long FLOPS_TRIE = " << em.trie_count.flops() << ";\n";
    h << "  static constexpr long FLOPS_REVERSE = " << cr.flops() << ";\n";
    h << "  static constexpr bool STAGED = true;\n";
    h << "  static constexpr int STAGE_G = " << STAGE_G << ", STAGE_R = " << STAGE_R << ";\n";
    h << "\n  template <typename T, bool WB, typename GP, typename XP, typename BP, typename DP>\n";
    h << "  __device__ __forceinline__ static void trie(GP gin, XP xi, BP Bout, DP dgout, T &V) {\n"
      << walk << "  }\n";
    h << "};\n";
    std::ofstream out(dir + "/mtp_level" + L + ".inc");
    out << h.str();
    std::cout << "level " << level << ": graphs " << B.graphs.size() << " basis " << B.n_lin() << " comps "
              << B.n_comp() << " flops graphs " << cf.flops() << " trie " << em.trie_count.flops() << " reverse "
              << cr.flops() << " (staged: " << STAGE_G << " graph parts, " << STAGE_R << " reverse parts)\n";
}

bool force_staged = false;   // --staged: every level as a staged program (for checking the two forms)
bool force_single = false;   // --single: every level as one program

void write_level(const std::string &dir, int level) {
    Basis B = build_basis(level);
    if (force_staged || (!force_single && (int)B.graphs.size() > STAGED_GRAPHS))
        return write_level_staged(dir, level, B);
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
    h << "  static constexpr bool STAGED = false;\n";
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
    for (int i = 2; i < argc; ++i) {
        if (std::string(argv[i]) == "--staged" || std::string(argv[i]) == "--single") {
            (argv[i][2] == 's' && argv[i][3] == 't' ? force_staged : force_single) = true;
            continue;
        }
        write_level(argv[1], std::atoi(argv[i]));
    }
    return 0;
}
