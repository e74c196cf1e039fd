"""Basis enumeration of the MTP (paper Sec. II.A, eqs. 5-6) -- oracle side.

Test infrastructure only (see ``oracle/__init__.py``).

The paper defines the level of a moment, lev M_{mu,nu} = 2 + 4 mu + nu (eq. 5),
the level of a product of moments as the sum of their levels (eq. 6), and
keeps every basis function whose level is at most lev_max.  It shows the
basis functions are full contractions of products of moments to a scalar
(examples M_{1,0}, (M_{1,2} M_{0,1}) . M_{0,1}, M_{1,2} : M_{3,2}) and lists
the level-6 set explicitly.  It does not state which contractions are
admitted.  Reading used here (it reproduces every count the paper prints:
N_lin = 5 and N_rad = 2 at level 6, and |theta| = 26 / 54 / 125 at levels
8 / 12 / 16 for one species):

* a contraction is a multigraph whose nodes are moments M_{mu,nu} (node
  degree = nu) and whose edges are contracted index pairs between two
  *different* moments (no self-contraction, i.e. no traces);
* at most two edges join any two nodes, and nu <= 3;
* a basis function is a multiset of connected contraction graphs, i.e. a
  product of scalar invariants; graphs are identified up to isomorphism
  preserving the node labels (mu, nu).

Canonical forms and the order of the basis (a convention, it only fixes the
column order of xi and of the rows b_i):

* a graph's nodes are sorted by label (mu, nu); among all node orders that
  keep the labels sorted, the canonical one has the lexicographically
  smallest tuple of edge multiplicities e_pq listed for p < q in row-major
  order;
* graph key   = (level, number of nodes, labels, edge tuple);
* a basis function's factors are sorted by graph key;
  basis key   = (level, number of factors, tuple of factor keys);
* the basis is sorted by basis key.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from functools import lru_cache

MAX_NU = 3          # rank bound of the reading above
MAX_MULT = 2        # edge multiplicity bound of the reading above


def moment_level(mu: int, nu: int) -> int:
    """lev M_{mu,nu} = 2 + 4 mu + nu (eq. 5)."""
    return 2 + 4 * mu + nu


@dataclass(frozen=True)
class Graph:
    """A connected contraction graph.

    labels : tuple of (mu, nu), sorted
    edges  : tuple of e_pq for p < q (row-major), canonical
    """

    labels: tuple
    edges: tuple

    @property
    def n(self) -> int:
        return len(self.labels)

    @property
    def level(self) -> int:
        return sum(moment_level(mu, nu) for mu, nu in self.labels)

    def key(self):
        return (self.level, self.n, self.labels, self.edges)

    def edge_list(self):
        """[(p, q, multiplicity)] with multiplicity > 0."""
        out, k = [], 0
        for p in range(self.n):
            for q in range(p + 1, self.n):
                if self.edges[k]:
                    out.append((p, q, self.edges[k]))
                k += 1
        return out

    def __str__(self):
        s = " ".join(f"M{mu}{nu}" for mu, nu in self.labels)
        e = ",".join(f"{p}-{q}:{m}" for p, q, m in self.edge_list())
        return f"[{s}]" + (f"({e})" if e else "")


def _pairs(n):
    return [(p, q) for p in range(n) for q in range(p + 1, n)]


def _edge_assignments(nus):
    """All symmetric multiplicity matrices with row sums nus, entries 0..MAX_MULT."""
    n = len(nus)
    pairs = _pairs(n)
    out = []

    def rec(k, rem, acc):
        if k == len(pairs):
            if all(r == 0 for r in rem):
                out.append(tuple(acc))
            return
        p, q = pairs[k]
        for m in range(0, min(MAX_MULT, rem[p], rem[q]) + 1):
            rem[p] -= m
            rem[q] -= m
            acc.append(m)
            rec(k + 1, rem, acc)
            acc.pop()
            rem[p] += m
            rem[q] += m

    rec(0, list(nus), [])
    return out


def _connected(n, edges):
    adj = {p: set() for p in range(n)}
    for (p, q), m in zip(_pairs(n), edges):
        if m:
            adj[p].add(q)
            adj[q].add(p)
    seen, stack = {0}, [0]
    while stack:
        for q in adj[stack.pop()]:
            if q not in seen:
                seen.add(q)
                stack.append(q)
    return len(seen) == n


def _canonical(labels, edges):
    """Smallest edge tuple over all label-preserving node permutations."""
    n = len(labels)
    mat = [[0] * n for _ in range(n)]
    for (p, q), m in zip(_pairs(n), edges):
        mat[p][q] = mat[q][p] = m
    best = None
    for perm in itertools.permutations(range(n)):
        if any(labels[perm[k]] != labels[k] for k in range(n)):
            continue
        cand = tuple(mat[perm[p]][perm[q]] for p, q in _pairs(n))
        if best is None or cand < best:
            best = cand
    return best


@lru_cache(maxsize=None)
def connected_graphs(lev_max: int):
    """Every connected contraction graph with level <= lev_max, sorted by key."""
    moments = [(mu, nu) for mu in range(lev_max) for nu in range(MAX_NU + 1)
               if moment_level(mu, nu) <= lev_max]
    found = set()
    # one node: must be a scalar moment (no self-contraction)
    for mu, nu in moments:
        if nu == 0:
            found.add(Graph(((mu, nu),), ()))
    # two or more nodes: every node needs an edge, so nu >= 1 everywhere
    tensors = [m for m in moments if m[1] >= 1]
    for n in range(2, lev_max // 3 + 1):
        for labels in itertools.combinations_with_replacement(sorted(tensors), n):
            if sum(moment_level(*m) for m in labels) > lev_max:
                continue
            for edges in _edge_assignments([nu for _, nu in labels]):
                if _connected(n, edges):
                    found.add(Graph(labels, _canonical(labels, edges)))
    return tuple(sorted(found, key=Graph.key))


@dataclass(frozen=True)
class BasisFunction:
    factors: tuple  # tuple of Graph, sorted by key

    @property
    def level(self):
        return sum(g.level for g in self.factors)

    def key(self):
        return (self.level, len(self.factors), tuple(g.key() for g in self.factors))

    def __str__(self):
        return "*".join(str(g) for g in self.factors)


@lru_cache(maxsize=None)
def basis(lev_max: int):
    """All products of connected graphs with total level <= lev_max (eq. 6), sorted."""
    graphs = connected_graphs(lev_max)
    out = []

    def extend(start, budget, combo):
        # multisets are generated as non-decreasing index sequences
        if combo:
            out.append(BasisFunction(tuple(sorted(combo, key=Graph.key))))
        for k in range(start, len(graphs)):
            if graphs[k].level <= budget:
                combo.append(graphs[k])
                extend(k, budget - graphs[k].level, combo)
                combo.pop()

    extend(0, lev_max, [])
    return tuple(sorted(out, key=BasisFunction.key))


def n_rad(lev_max: int) -> int:
    """Number of radial functions: largest mu occurring in the basis, plus one."""
    return 1 + max(mu for b in basis(lev_max) for g in b.factors for mu, _ in g.labels)


def moments_used(lev_max: int):
    """Sorted list of the (mu, nu) that occur in the basis."""
    return sorted({lab for b in basis(lev_max) for g in b.factors for lab in g.labels})


def n_params(lev_max: int, n_types: int, n_polyn: int = 8) -> int:
    """|theta| = N_types (species constants) + N_lin + N_polyn * N_rad * N_types^2 (eq. 4)."""
    return n_types + len(basis(lev_max)) + n_polyn * n_rad(lev_max) * n_types ** 2
