"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numbers the
paper prints (tests/golden/paper_facts.json), closed forms, brute-force sums,
invariances, finite differences and exhaustive searches.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import basis as ob
from oracle import mtp as om
from oracle import neighbors as onb

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def _bcc(reps=(2, 2, 2), a=3.3, sigma=0.1, seed=0):
    base = np.array([[0, 0, 0], [0.5, 0.5, 0.5]])
    g = np.array([[i, j, k] for i in range(reps[0]) for j in range(reps[1]) for k in range(reps[2])])
    pos = (g[:, None, :] + base[None]).reshape(-1, 3) * a
    pos = pos + np.random.default_rng(seed).normal(0, sigma, pos.shape)
    return pos, np.diag(np.asarray(reps, float) * a)


def _name(bf):
    parts = []
    for g in bf.factors:
        if g.n == 1:
            parts.append("M%d%d" % g.labels[0])
        elif g.n == 2 and g.edges == (1,):
            parts.append("M%d%d.M%d%d" % (g.labels[0] + g.labels[1]))
        else:
            parts.append(str(g))
    out = []
    for p, grp in itertools.groupby(parts):
        k = len(list(grp))
        out.append(p if k == 1 else f"{p}^{k}")
    return "*".join(out)


# ---------------------------------------------------------------- basis ----
def test_moment_level_examples():
    for mu, nu, lev in GOLD["moment_level_examples"]["values"]:
        assert ob.moment_level(mu, nu) == lev


def test_level6_basis_matches_paper():
    names = sorted(_name(b) for b in ob.basis(6))
    assert names == sorted(GOLD["level6_basis"]["functions"])
    assert len(ob.basis(6)) == GOLD["level6_basis"]["n_lin"]
    assert ob.n_rad(6) == GOLD["level6_basis"]["n_rad"]


def test_parameter_counts_match_paper():
    for lev, n in GOLD["n_params_one_species"]["values"].items():
        assert ob.n_params(int(lev), 1) == n


def test_contraction_examples_are_basis_members():
    for ex in GOLD["contraction_examples"]["graphs"]:
        labels = tuple(tuple(l) for l in ex["labels"])
        lev = sum(ob.moment_level(*l) for l in labels)
        found = [g for g in ob.connected_graphs(lev) if g.labels == labels]
        want = sorted((p, q, m) for p, q, m in ex["edges"])
        assert any(sorted(g.edge_list()) == want for g in found), ex
        # and it is absent one level below
        assert not any(g.labels == labels for g in ob.connected_graphs(lev - 1))


def test_basis_closed_under_isomorphism_dedup():
    # a graph and a relabelled copy must not both occur
    for g in ob.connected_graphs(16):
        assert g.edges == ob._canonical(g.labels, g.edges)
    keys = [b.key() for b in ob.basis(16)]
    assert len(keys) == len(set(keys))


# --------------------------------------------------------------- radial ----
def test_chebyshev_is_cos_k_t():
    t = torch.linspace(0.0, math.pi, 37, dtype=torch.float64)
    T = om.chebyshev(torch.cos(t), 8)
    for k in range(8):
        assert torch.allclose(T[:, k], torch.cos(k * t), atol=1e-13)


def test_radial_vanishes_smoothly_at_cutoff():
    pot = om.Potential(8, 2, 2.0, 5.0)
    c = torch.as_tensor(np.random.default_rng(1).normal(size=(pot.n_rad, 2, 2, 8)))
    r = torch.tensor([5.0, 5.0 - 1e-6], dtype=torch.float64)
    f = om.radial_functions(pot, c, r, torch.tensor([0, 1]), torch.tensor([1, 1]))
    assert torch.all(f[0] == 0)
    assert torch.all(f[1].abs() < 1e-10)        # quadratic zero: f ~ (R_cut - r)^2


def test_radial_at_rmin_is_plain_sum():
    # at r = R_min, x = -1 and T_k(-1) = (-1)^k, so f = (R_cut - R_min)^2 sum_b c_b (-1)^(b-1)
    pot = om.Potential(8, 1, 2.0, 5.0)
    c = torch.as_tensor(np.random.default_rng(2).normal(size=(pot.n_rad, 1, 1, 8)))
    f = om.radial_functions(pot, c, torch.tensor([2.0], dtype=torch.float64), torch.tensor([0]), torch.tensor([0]))
    sign = torch.tensor([(-1.0) ** k for k in range(8)], dtype=torch.float64)
    want = 9.0 * (c[:, 0, 0, :] * sign).sum(-1)
    assert torch.allclose(f[0], want, rtol=1e-13)


# --------------------------------------------------------- contractions ----
def _pair_sum_value(g, f, R):
    """val(G) = sum over one neighbor per node of prod f * prod (r_p . r_q)^e."""
    n = len(R)
    total = 0.0
    for js in itertools.product(range(n), repeat=g.n):
        v = 1.0
        for p, (mu, _) in enumerate(g.labels):
            v *= f[js[p], mu]
        for p, q, m in g.edge_list():
            v *= float(np.dot(R[js[p]], R[js[q]])) ** m
        total += v
    return total


@pytest.mark.parametrize("level", [16])
def test_graph_values_equal_brute_force_pair_sums(level):
    rng = np.random.default_rng(3)
    R = rng.normal(size=(3, 3))
    f = rng.normal(size=(3, 4))
    Rt = torch.as_tensor(R)
    ft = torch.as_tensor(f)
    M = {}
    for mu in range(4):
        M[(mu, 0)] = ft[:, mu].sum()[None]
        M[(mu, 1)] = torch.einsum("p,pa->a", ft[:, mu], Rt)[None]
        M[(mu, 2)] = torch.einsum("p,pa,pb->ab", ft[:, mu], Rt, Rt)[None]
        M[(mu, 3)] = torch.einsum("p,pa,pb,pc->abc", ft[:, mu], Rt, Rt, Rt)[None]
    for g in ob.connected_graphs(level):
        got = float(om.graph_value(g, M)[0])
        want = _pair_sum_value(g, f, R)
        assert abs(got - want) <= 1e-11 * max(1.0, abs(want)), str(g)


def test_closed_forms():
    rng = np.random.default_rng(4)
    R = torch.as_tensor(rng.normal(size=(5, 3)))
    f = torch.as_tensor(rng.normal(size=5))
    M01 = (f[:, None] * R).sum(0)[None]
    M02 = torch.einsum("p,pa,pb->ab", f, R, R)[None]
    g11 = [g for g in ob.connected_graphs(6) if g.labels == ((0, 1), (0, 1))][0]
    g22 = [g for g in ob.connected_graphs(8) if g.labels == ((0, 2), (0, 2))][0]
    g222 = [g for g in ob.connected_graphs(12) if g.labels == ((0, 2),) * 3][0]
    M = {(0, 1): M01, (0, 2): M02}
    assert torch.allclose(om.graph_value(g11, M), (M01 ** 2).sum(), rtol=1e-13)
    G = R @ R.T
    assert torch.allclose(om.graph_value(g22, M), (f[:, None] * f[None] * G ** 2).sum(), rtol=1e-12)
    assert torch.allclose(om.graph_value(g222, M), torch.trace(M02[0] @ M02[0] @ M02[0]), rtol=1e-12)


# ------------------------------------------------------------- moments -----
def _cheb_closed(x, k):
    """T_k(x) from its trigonometric / hyperbolic closed form (no recurrence)."""
    if abs(x) <= 1.0:
        return math.cos(k * math.acos(x))
    return math.cosh(k * math.acosh(abs(x))) * (math.copysign(1.0, x) ** k)


def _radial_by_hand(c, r, zi, zj, r_min=2.0, r_cut=5.0):
    """f_mu(r) = sum_beta c[mu, zi, zj, beta] T_beta(x) (R_cut - r)^2 (eq. 4), written out."""
    x = (2.0 * r - r_min - r_cut) / (r_cut - r_min)
    return [sum(c[mu, zi, zj, b] * _cheb_closed(x, b) for b in range(c.shape[3])) * (r_cut - r) ** 2
            for mu in range(c.shape[0])]


def _tiny_neighborhoods(seed, n_atoms=3, n_nbrs=(3, 4, 2)):
    """Free pairs (no lattice): n_nbrs[i] neighbors of atom i at random directions, 2.1-4.9 A."""
    rng = np.random.default_rng(seed)
    rv, ii, jj = [], [], []
    for i in range(n_atoms):
        for _ in range(n_nbrs[i]):
            d = rng.normal(size=3)
            rv.append(d / np.linalg.norm(d) * rng.uniform(2.1, 4.9))
            ii.append(i)
            jj.append(int(rng.integers(0, n_atoms)))
    return np.array(rv), np.array(ii), np.array(jj)


def test_moments_equal_explicit_monomial_loops():
    """M_{mu,nu}[a1..anu] = sum_j f_mu(|r_ij|) r_ij[a1] ... r_ij[anu] (eq. 3) by plain loops over
    neighbors and index tuples, for every (mu, nu) of level 16 with two species (mu <= 3, nu <= 3)."""
    pot = om.Potential(16, 2, 2.0, 5.0)
    rng = np.random.default_rng(11)
    c = rng.normal(size=(pot.n_rad, 2, 2, 8))
    types = np.array([0, 1, 1])
    rv, ii, jj = _tiny_neighborhoods(12)
    M = om.moments(pot, torch.as_tensor(c), torch.as_tensor(rv), torch.as_tensor(ii),
                   torch.as_tensor(types[ii]), torch.as_tensor(types[jj]), 3)
    assert {nu for _, nu in pot.moments} == {0, 1, 2, 3} and {mu for mu, _ in pot.moments} == {0, 1, 2, 3}
    for mu, nu in pot.moments:
        got = M[(mu, nu)].numpy()
        for i in range(3):
            for idx in itertools.product(range(3), repeat=nu):
                want = 0.0
                for p in np.where(ii == i)[0]:
                    f = _radial_by_hand(c, float(np.linalg.norm(rv[p])), types[i], types[jj[p]])[mu]
                    term = f
                    for a in idx:
                        term *= rv[p][a]
                    want += term
                assert abs(got[(i,) + idx] - want) <= 1e-12 * max(1.0, abs(want)), (mu, nu, i, idx)


def test_moments_single_neighbor_closed_form():
    """One neighbor at (d, 0, 0): M_{mu,1} = f_mu(d) d e_x, M_{mu,2} = f_mu(d) d^2 e_x e_x,
    M_{mu,3}[0,0,0] = f_mu(d) d^3 and every other entry zero."""
    pot = om.Potential(16, 1, 2.0, 5.0)
    c = np.random.default_rng(13).normal(size=(pot.n_rad, 1, 1, 8))
    for d in (2.3, 3.7, 4.6):
        M = om.moments(pot, torch.as_tensor(c), torch.tensor([[d, 0.0, 0.0]], dtype=torch.float64),
                       torch.tensor([0]), torch.tensor([0]), torch.tensor([0]), 1)
        f = _radial_by_hand(c, d, 0, 0)
        for mu, nu in pot.moments:
            want = np.zeros((3,) * nu)
            want[(0,) * nu] = f[mu] * d ** nu
            assert np.allclose(M[(mu, nu)].numpy()[0], want, rtol=1e-13, atol=1e-13 * abs(f[mu]) * d ** nu)


def test_site_energies_equal_pair_sum_basis():
    """V_i = xi_0[z_i] + sum_alpha xi_alpha prod_{G in alpha} val(G) (eq. 2) with every graph value
    written as the pair sum over one neighbor per node of prod f_mu(|r_j|) prod (r_p . r_q)^e:
    raw r_ij (not unit vectors) and a hand-written radial, through om.site_energies."""
    pot = om.Potential(12, 2, 2.0, 5.0)
    rng = np.random.default_rng(14)
    theta = rng.normal(0, 0.3, pot.n_theta)
    xi0, xi, c = theta[:2], theta[2:2 + pot.n_lin], theta[2 + pot.n_lin:].reshape(pot.n_rad, 2, 2, 8)
    types = np.array([1, 0, 1])
    rv, ii, jj = _tiny_neighborhoods(15, n_nbrs=(3, 2, 4))
    V, _ = om.site_energies(pot, torch.as_tensor(theta), torch.as_tensor(rv), torch.as_tensor(ii),
                            torch.as_tensor(jj), types, 3)
    for i in range(3):
        ps = np.where(ii == i)[0]
        R = rv[ps]
        f = np.array([_radial_by_hand(c, float(np.linalg.norm(r)), types[i], types[jj[p]]) for r, p in zip(R, ps)])
        gv = {}
        want = xi0[types[i]]
        for a, bf in enumerate(pot.basis):
            v = 1.0
            for g in bf.factors:
                if g not in gv:
                    gv[g] = _pair_sum_value(g, f, R)
                v *= gv[g]
            want += xi[a] * v
        assert abs(float(V[i]) - want) <= 1e-11 * max(1.0, abs(want)), (i, float(V[i]), want)


# -------------------------------------------------------------- energy -----
def _nbrs(pos, cell, pbc=(1, 1, 1), rc=5.0):
    return onb.neighbors(pos, cell, pbc, rc)


def test_level2_is_pair_potential():
    pos, cell = _bcc()
    pot = om.Potential(2, 1, 2.0, 5.0)
    theta = np.random.default_rng(5).normal(0, 0.1, pot.n_theta)
    pairs = _nbrs(pos, cell)
    E, F, S, V = om.energy_forces_stress(pot, theta, pos, np.zeros(len(pos), int), cell, pairs)
    xi0, xi, c = theta[0], theta[1], theta[2:]
    want = 0.0
    for i in range(len(pos)):
        vi = xi0
        for p in np.where(pairs.i == i)[0]:
            r = np.linalg.norm(pos[pairs.j[p]] + pairs.shift[p] @ cell - pos[i])
            x = (2 * r - 7.0) / 3.0
            T = [math.cos(k * math.acos(x)) if abs(x) <= 1 else math.cosh(k * math.acosh(abs(x))) * (np.sign(x) ** k)
                 for k in range(8)]
            vi += xi * sum(c[b] * T[b] for b in range(8)) * (5.0 - r) ** 2
        want += vi
    assert abs(E - want) <= 1e-11 * abs(want)


def test_level4_is_quadratic_embedding():
    pos, cell = _bcc(sigma=0.05)
    pot = om.Potential(4, 1, 2.0, 5.0)
    theta = np.random.default_rng(6).normal(0, 0.1, pot.n_theta)
    pairs = _nbrs(pos, cell)
    E, F, S, V = om.energy_forces_stress(pot, theta, pos, np.zeros(len(pos), int), cell, pairs)
    c = torch.as_tensor(theta[3:]).reshape(1, 1, 1, 8)
    rv = torch.as_tensor(pos[pairs.j] + pairs.shift @ cell - pos[pairs.i])
    f = om.radial_functions(pot, c, torch.linalg.norm(rv, dim=1), torch.zeros(len(rv), dtype=torch.long),
                            torch.zeros(len(rv), dtype=torch.long))[:, 0].numpy()
    rho = np.bincount(pairs.i, weights=f, minlength=len(pos))
    want = theta[0] + theta[1] * rho + theta[2] * rho ** 2
    assert np.allclose(V, want, rtol=1e-12, atol=1e-12)


def _setup(level=8, n_types=2, seed=7, reps=(2, 2, 2), sigma=0.1):
    pos, cell = _bcc(reps, sigma=sigma, seed=seed)
    types = np.random.default_rng(seed + 1).integers(0, n_types, len(pos))
    pot = om.Potential(level, n_types, 2.0, 5.0)
    theta = np.random.default_rng(seed + 2).normal(0, 0.1, pot.n_theta)
    return pot, theta, pos, types, cell


def _random_rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_invariances_translation_rotation_permutation():
    pot, theta, pos, types, cell = _setup(level=12)
    E0, F0, S0, V0 = om.energy_forces_stress(pot, theta, pos, types, cell, _nbrs(pos, cell))
    # translation
    p1 = pos + np.array([0.37, -1.2, 2.5])
    E1, F1, _, V1 = om.energy_forces_stress(pot, theta, p1, types, cell, _nbrs(p1, cell))
    assert abs(E1 - E0) <= 1e-10 * abs(E0) and np.allclose(F1, F0, atol=1e-9 * np.abs(F0).max())
    # rotation of positions and cell together
    Q = _random_rotation(11)
    p2, c2 = pos @ Q.T, cell @ Q.T
    E2, F2, S2, _ = om.energy_forces_stress(pot, theta, p2, types, c2, _nbrs(p2, c2))
    assert abs(E2 - E0) <= 1e-10 * abs(E0)
    assert np.allclose(F2, F0 @ Q.T, atol=1e-9 * np.abs(F0).max())
    assert np.allclose(S2, Q @ S0 @ Q.T, atol=1e-9 * np.abs(S0).max())
    # permutation of atoms
    perm = np.random.default_rng(12).permutation(len(pos))
    p3, t3 = pos[perm], types[perm]
    E3, F3, _, V3 = om.energy_forces_stress(pot, theta, p3, t3, cell, _nbrs(p3, cell))
    assert abs(E3 - E0) <= 1e-10 * abs(E0)
    assert np.allclose(F3, F0[perm], atol=1e-9 * np.abs(F0).max())
    assert np.allclose(V3, V0[perm], rtol=1e-10, atol=1e-10 * np.abs(V0).max())


def test_additivity_of_separated_clusters():
    pot = om.Potential(12, 1, 2.0, 5.0)
    theta = np.random.default_rng(13).normal(0, 0.1, pot.n_theta)
    rng = np.random.default_rng(14)
    a = rng.normal(0, 1.5, (5, 3))
    b = rng.normal(0, 1.5, (4, 3)) + np.array([40.0, 0, 0])
    cell = np.eye(3) * 100.0
    pbc = (0, 0, 0)
    t = np.zeros(9, int)
    Ea = om.energy_forces_stress(pot, theta, a, t[:5], cell, onb.neighbors(a, cell, pbc, 5.0))[0]
    Eb = om.energy_forces_stress(pot, theta, b, t[:4], cell, onb.neighbors(b, cell, pbc, 5.0))[0]
    ab = np.vstack([a, b])
    Eab = om.energy_forces_stress(pot, theta, ab, t, cell, onb.neighbors(ab, cell, pbc, 5.0))[0]
    assert abs(Eab - (Ea + Eb)) <= 1e-12 * (abs(Ea) + abs(Eb))


# ------------------------------------------------------ forces / stress ----
def test_forces_and_stress_match_finite_differences():
    pot, theta, pos, types, cell = _setup(level=12, sigma=0.12)
    pairs = _nbrs(pos, cell)
    E, F, S, _ = om.energy_forces_stress(pot, theta, pos, types, cell, pairs)
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.abs(F).max()
    assert np.allclose(S, S.T, atol=1e-10 * np.abs(S).max())
    h = 1e-5
    for (i, k) in [(0, 0), (3, 1), (7, 2), (12, 0)]:
        # the pair set does not change for this small step (no pair sits at R_cut)
        pp, pm = pos.copy(), pos.copy()
        pp[i, k] += h
        pm[i, k] -= h
        Ep = om.energy_forces_stress(pot, theta, pp, types, cell, pairs)[0]
        Em = om.energy_forces_stress(pot, theta, pm, types, cell, pairs)[0]
        fd = -(Ep - Em) / (2 * h)
        assert abs(fd - F[i, k]) <= 1e-7 * np.abs(F).max(), (i, k, fd, F[i, k])
    hs = 1e-6
    for (a, b) in [(0, 0), (0, 1), (2, 1), (2, 2)]:
        D = np.zeros((3, 3))
        D[a, b] = hs
        Ep = om.energy_forces_stress(pot, theta, pos @ (np.eye(3) + D).T, types, cell @ (np.eye(3) + D).T, pairs)[0]
        Em = om.energy_forces_stress(pot, theta, pos @ (np.eye(3) - D).T, types, cell @ (np.eye(3) - D).T, pairs)[0]
        fd = -(Ep - Em) / (2 * hs)
        assert abs(fd - S[a, b]) <= 1e-6 * np.abs(S).max(), (a, b, fd, S[a, b])


# -------------------------------------------------------------- b rows -----
def _n_factors_moments(pot):
    return np.array([sum(g.n for g in bf.factors) for bf in pot.basis])


def test_b_rows_match_finite_differences_and_euler_identity():
    pot, theta, pos, types, cell = _setup(level=8)
    pairs = _nbrs(pos, cell)
    b = om.b_rows(pot, theta, pos, types, cell, pairs)
    h = 1e-6
    for p in [0, 1, 2, 5, pot.n_types + pot.n_lin, pot.n_theta - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        Vp = om.energy_forces_stress(pot, tp, pos, types, cell, pairs)[3]
        Vm = om.energy_forces_stress(pot, tm, pos, types, cell, pairs)[3]
        assert np.allclose((Vp - Vm) / (2 * h), b[:, p], atol=1e-6 * np.abs(b[:, p]).max() + 1e-9)
    # Euler: B_alpha is homogeneous of degree P_alpha (number of moment factors) in c
    _, _, V = om.energy_forces_stress(pot, theta, pos, types, cell, pairs)[1:]
    lin = om.linear_rows(pot, theta, pos, types, cell, pairs)
    B = lin[:, pot.n_types:]
    xi0, xi = theta[:pot.n_types], theta[pot.n_types:pot.n_types + pot.n_lin]
    want = xi0[types] + B @ ((1 + _n_factors_moments(pot)) * xi)
    assert np.allclose(b @ theta, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())
    assert np.allclose(xi0[types] + B @ xi, V, rtol=1e-12, atol=1e-12 * np.abs(V).max())


def _null_vectors(pot, theta):
    """w_{mu mu'}: remix f_mu += t f_mu' (mu' <= mu), compensated by xi."""
    T, L = pot.n_types, pot.n_lin
    c = theta[T + L:].reshape(pot.n_rad, -1)
    out = []
    for mu in range(pot.n_rad):
        for mup in range(mu + 1):
            w = np.zeros(pot.n_theta)
            w[T + L + mu * c.shape[1]: T + L + (mu + 1) * c.shape[1]] = c[mup]
            for a, bf in enumerate(pot.basis):
                # each occurrence of a mu-moment turns into a mu'-moment: the
                # resulting product is again a basis function, whose xi absorbs it
                for gi, g in enumerate(bf.factors):
                    for ni, (m, nu) in enumerate(g.labels):
                        if m != mu:
                            continue
                        labels = list(g.labels)
                        labels[ni] = (mup, nu)
                        tgt = _find_basis(pot, bf, gi, ni, mup)
                        w[T + tgt] -= theta[T + a]
            out.append(w)
    return np.array(out)


def _find_basis(pot, bf, gi, ni, mup):
    g = bf.factors[gi]
    labels = list(g.labels)
    labels[ni] = (mup, labels[ni][1])
    # canonicalise the relabelled graph by brute force over all node orders
    n = g.n
    mat = np.zeros((n, n), int)
    for p, q, m in g.edge_list():
        mat[p, q] = mat[q, p] = m
    best = None
    for perm in itertools.permutations(range(n)):
        lab = tuple(labels[k] for k in perm)
        if list(lab) != sorted(lab):
            continue
        e = tuple(mat[perm[p], perm[q]] for p in range(n) for q in range(p + 1, n))
        if best is None or e < best[1]:
            best = (lab, e)
    newg = ob.Graph(best[0], best[1])
    factors = list(bf.factors)
    factors[gi] = newg
    key = ob.BasisFunction(tuple(sorted(factors, key=ob.Graph.key))).key()
    keys = [b.key() for b in pot.basis]
    return keys.index(key)


def test_b_rows_null_space_and_rank():
    pot, theta, pos, types, cell = _setup(level=8, n_types=2, reps=(3, 3, 3))
    rows = []
    for seed in range(3):
        p, _ = _bcc((3, 3, 3), sigma=0.25, seed=100 + seed)
        rows.append(om.b_rows(pot, theta, p, types, cell, _nbrs(p, cell)))
    b = np.vstack(rows)
    W = _null_vectors(pot, theta)
    assert W.shape[0] == pot.n_rad * (pot.n_rad + 1) // 2
    assert np.abs(b @ W.T).max() <= 1e-11 * np.abs(b).max() * np.abs(W).max()
    sv = np.linalg.svd(b / np.abs(b).max(0), compute_uv=False)
    rank = int((sv > 1e-9 * sv[0]).sum())
    assert rank == pot.n_theta - W.shape[0]
    # gauge-fixed columns have full rank
    keep = om.kept_columns(pot, theta)
    sv2 = np.linalg.svd(b[:, keep] / np.abs(b[:, keep]).max(0), compute_uv=False)
    assert sv2[-1] > 1e-9 * sv2[0]


# -------------------------------------------------------------- grades -----
def _active_case(level=8, n_types=1, reps=(3, 3, 3), seed=21):
    pot, theta, pos, types, cell = _setup(level=level, n_types=n_types, reps=reps, seed=seed)
    pairs = _nbrs(pos, cell)
    keep = om.kept_columns(pot, theta)
    b = om.b_rows(pot, theta, pos, types, cell, pairs)[:, keep]
    act = om.initial_active_set(b)
    return pot, theta, pos, types, cell, pairs, keep, b, act


def test_gamma_is_one_on_active_rows_and_scale_invariant():
    pot, theta, pos, types, cell, pairs, keep, b, act = _active_case()
    A = b[act]
    g, am, _ = om.grades(A, A)
    assert np.allclose(g, 1.0, atol=1e-12)
    assert np.array_equal(am, np.arange(len(act)))
    D = np.diag(np.random.default_rng(22).uniform(0.1, 10, A.shape[1]))
    g1, _, _ = om.grades(b, A)
    g2, _, _ = om.grades(b @ D, A @ D)
    assert np.allclose(g1, g2, rtol=1e-9)


def test_gamma_independent_of_gauge_choice():
    pot, theta, pos, types, cell = _setup(level=8, n_types=1, reps=(3, 3, 3), seed=23)
    pairs = _nbrs(pos, cell)
    full = om.b_rows(pot, theta, pos, types, cell, pairs)
    keep1 = om.kept_columns(pot, theta)
    # another valid gauge: drop different columns of each c block
    T, L = pot.n_types, pot.n_lin
    c = theta[T + L:].reshape(pot.n_rad, -1)
    drop2 = []
    for mu in range(pot.n_rad):
        cols = list(range(c.shape[1] - 1, -1, -1))[: mu + 1]
        assert abs(np.linalg.det(c[: mu + 1][:, cols])) > 1e-8
        drop2 += [T + L + mu * c.shape[1] + k for k in cols]
    keep2 = [k for k in range(pot.n_theta) if k not in drop2]
    assert keep1 != keep2
    act = om.initial_active_set(full[:, keep1])
    g1, _, _ = om.grades(full[:, keep1], full[act][:, keep1])
    g2, _, _ = om.grades(full[:, keep2], full[act][:, keep2])
    assert np.allclose(g1, g2, rtol=1e-7)


def test_gamma_rotation_invariant():
    pot, theta, pos, types, cell, pairs, keep, b, act = _active_case(seed=24)
    Q = _random_rotation(25)
    p2, c2 = pos @ Q.T, cell @ Q.T
    b2 = om.b_rows(pot, theta, p2, types, c2, _nbrs(p2, c2))[:, keep]
    g1, _, _ = om.grades(b, b[act])
    g2, _, _ = om.grades(b2, b2[act])
    assert np.allclose(g1, g2, rtol=1e-8)


def test_linear_mode_reproduces_site_energies():
    # with the active set as training set, V_i = sum_j c_ij V(n_j^act) (linear case)
    pot, theta, pos, types, cell = _setup(level=8, n_types=2, reps=(3, 3, 3), seed=26)
    pairs = _nbrs(pos, cell)
    lin = om.linear_rows(pot, theta, pos, types, cell, pairs)
    V = om.energy_forces_stress(pot, theta, pos, types, cell, pairs)[3]
    act = om.initial_active_set(lin)
    _, _, C = om.grades(lin, lin[act])
    assert np.allclose(C @ V[act], V, rtol=1e-9, atol=1e-9 * np.abs(V).max())


# ------------------------------------------------- configuration mode -----
def _small_cfgs(n_cfg, seed, n_types=1, level=8):
    """Small BCC cells (2x2x2 or 3x2x2) with random vacancies and species."""
    r = np.random.default_rng(seed)
    out = []
    for k in range(n_cfg):
        reps = (2, 2, 2) if k % 2 == 0 else (3, 2, 2)
        pos, cell = _bcc(reps, sigma=0.12, seed=seed * 1000 + k)
        keep = np.sort(r.choice(len(pos), len(pos) - int(r.integers(0, 4)), replace=False))
        types = r.integers(0, n_types, len(keep)).astype(np.int32)
        out.append((pos[keep], types, cell))
    return out


def test_cfg_rows_are_total_energy_gradients():
    # b(cfg) = dE(cfg)/dtheta (Sec. II.C): central differences of the total energy
    pot, theta, _, _, _ = _setup(level=8, n_types=2)
    (pos, types, cell), = _small_cfgs(1, 41, n_types=2)
    pairs = _nbrs(pos, cell)
    b = om.cfg_rows(om.b_rows(pot, theta, pos, types, cell, pairs), [len(pos)])[0]
    h = 1e-6
    for p in [0, 1, 2, 7, pot.n_types + pot.n_lin, pot.n_types + pot.n_lin + 9, pot.n_theta - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        Ep = om.energy_forces_stress(pot, tp, pos, types, cell, pairs)[0]
        Em = om.energy_forces_stress(pot, tm, pos, types, cell, pairs)[0]
        assert abs((Ep - Em) / (2 * h) - b[p]) <= 1e-6 * max(1.0, abs(b[p]))
    # the species columns count the atoms of each species
    assert np.array_equal(b[:pot.n_types], np.bincount(types, minlength=pot.n_types).astype(float))


def test_cfg_mode_linear_energies_are_combinations_of_active_energies():
    # with the active configurations as training set, E(cfg) = sum_j c_j E(cfg_j)
    # and c = b(cfg) A^-1 (Sec. II.C), exactly in the LINEAR mode
    pot, theta, _, _, _ = _setup(level=8, n_types=1)
    cfgs = _small_cfgs(24, 43)
    rows, E = [], []
    for pos, types, cell in cfgs:
        pairs = _nbrs(pos, cell)
        rows.append(om.cfg_rows(om.linear_rows(pot, theta, pos, types, cell, pairs), [len(pos)])[0])
        E.append(om.energy_forces_stress(pot, theta, pos, types, cell, pairs)[0])
    rows, E = np.array(rows), np.array(E)
    act = om.initial_active_set(rows)
    g, _, C = om.grades(rows, rows[act])
    assert np.allclose(g[act], 1.0, rtol=0, atol=1e-9)
    assert np.allclose(C @ E[act], E, rtol=1e-9, atol=1e-9 * np.abs(E).max())


# ------------------------------------- extrapolation-controlled runs -----
def test_neighborhood_cut_on_simple_cubic_shells():
    # shells of a simple cubic lattice: 1 + 6 (a), + 12 (sqrt 2 a), + 8 (sqrt 3 a)
    from oracle import al
    a = 2.5
    g = np.array([[i, j, k] for i in range(4) for j in range(4) for k in range(4)], float) * a
    cell = np.eye(3) * 4 * a
    grades = np.zeros(len(g))
    grades[21] = 3.0
    for cut, n in [(1.01 * a, 7), (1.42 * a, 19), (1.74 * a, 27)]:
        c, src, shift, p, _ = al.extrapolative_neighborhood(g, np.zeros(len(g), int), cell, (1, 1, 1), grades, cut)
        assert c == 21 and len(src) == n
        d = np.linalg.norm(p - g[21], axis=1)
        assert d.max() < cut and np.isclose(np.sort(d)[1], a)
    # ties: the lowest index
    assert al.extrapolative_neighborhood(g, np.zeros(len(g), int), cell, (1, 1, 1), np.ones(len(g)), 1.01 * a)[0] == 0


def _md_case():
    pot, theta, pos, types, cell = _setup(level=8, n_types=2, sigma=0.05)
    theta = theta.copy()
    theta[:pot.n_types + pot.n_lin] *= 1e-4   # E is linear in xi: forces of ~1 eV/A instead of ~1e4
    vel = np.random.default_rng(50).normal(0, 0.01, pos.shape)   # A/fs
    return pot, theta, pos, types, cell, vel, np.array([60.0, 30.0])


def test_md_verlet_is_time_reversible():
    from oracle import al
    pot, theta, pos, types, cell, vel, masses = _md_case()
    fw = al.md_verlet(pot, theta, pos, vel, types, cell, (1, 1, 1), masses, 1.0, 12, None, "full", None, 0, 1e300)
    bw = al.md_verlet(pot, theta, fw["pos"], -fw["vel"], types, cell, (1, 1, 1), masses, 1.0, 12, None, "full",
                      None, 0, 1e300)
    assert np.abs(fw["pos"] - pos).max() > 1e-3
    assert np.abs(bw["pos"] - pos).max() < 1e-10 and np.abs(bw["vel"] + vel).max() < 1e-12


def test_md_verlet_energy_error_is_second_order():
    from oracle import al
    pot, theta, pos, types, cell, vel, masses = _md_case()
    m_at = masses[types]

    def drift(dt, steps):
        x, v, worst = pos, vel, 0.0
        E0 = None
        for _ in range(steps):
            r = al.md_verlet(pot, theta, x, v, types, cell, (1, 1, 1), masses, dt, 1, None, "full", None, 0, 1e300)
            x, v = r["pos"], r["vel"]
            Ep = om.energy_forces_stress(pot, theta, x, types, cell, _nbrs(x, cell))[0]
            Ek = 0.5 * float((m_at[:, None] * v * v).sum()) / al.EV_PER_A_AMU_IN_A_PER_FS2
            E0 = (Ep + Ek) if E0 is None else E0
            worst = max(worst, abs(Ep + Ek - E0))
        return worst

    e1, e2 = drift(2.0, 8), drift(1.0, 16)
    assert 2.5 < e1 / e2 < 6.0


# ----------------------------------------------------------- fitting -----
def test_bfgs_minimizes_a_quadratic_and_rosenbrock():
    from oracle import fit
    r = np.random.default_rng(70)
    Q = r.normal(size=(6, 6))
    Q = Q @ Q.T + 6 * np.eye(6)
    b = r.normal(size=6)
    x, hist = fit.bfgs(lambda x: (0.5 * x @ Q @ x - b @ x, Q @ x - b), np.zeros(6), 100, gtol=1e-12)
    assert np.allclose(x, np.linalg.solve(Q, b), rtol=0, atol=1e-9)
    assert all(h1 <= h0 for h0, h1 in zip(hist, hist[1:]))

    def rosen(x):
        f = (1 - x[0]) ** 2 + 100 * (x[1] - x[0] ** 2) ** 2
        g = np.array([-2 * (1 - x[0]) - 400 * x[0] * (x[1] - x[0] ** 2), 200 * (x[1] - x[0] ** 2)])
        return f, g
    x, hist = fit.bfgs(rosen, np.array([-1.2, 1.0]), 500, gtol=1e-10)
    assert np.allclose(x, [1.0, 1.0], atol=1e-6) and hist[-1] < 1e-12


def test_bfgs_scale_is_a_change_of_variables():
    # H_0 = diag(D^2) on x gives the iterates of H_0 = I on u = x / D
    from oracle import fit
    D = np.array([1e3, 1.0, 1e-3])
    Q = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 3.0]])
    b = np.array([1.0, -2.0, 0.5])

    def fu(u):   # the quadratic in u
        return 0.5 * u @ Q @ u - b @ u, Q @ u - b

    def fx(x):   # the same function of x = D u
        u = x / D
        f, gu = fu(u)
        return f, gu / D
    u, hu = fit.bfgs(fu, np.zeros(3), 8, gtol=0)
    x, hx = fit.bfgs(fx, np.zeros(3), 8, gtol=0, scale=D)
    assert np.allclose(hx, hu, rtol=1e-9, atol=1e-14)
    assert np.allclose(x / D, u, rtol=1e-8, atol=1e-12)


def test_fire_finds_the_minimum_of_a_harmonic_well_and_stays_there():
    # F = -k (x - x0) per atom (k in eV/A^2): FIRE must end at x0; started
    # there, it takes no step
    from oracle import al
    r = np.random.default_rng(52)
    x0 = r.normal(0, 3.0, (20, 3))
    k = r.uniform(0.5, 5.0, 20)[:, None]
    inv_m = 1.0 / r.uniform(1.0, 200.0, 20)
    out = al.fire(x0 + r.normal(0, 0.3, x0.shape), inv_m, lambda x: -k * (x - x0), lambda x: 0.0, 1.0, 10.0, 1e-6,
                  5000, 2.0, 10.0)
    assert out["converged"] and np.abs(out["pos"] - x0).max() < 1e-6 / k.min()
    again = al.fire(x0, inv_m, lambda x: -k * (x - x0), lambda x: 0.0, 1.0, 10.0, 1e-6, 10, 2.0, 10.0)
    assert again["converged"] and again["steps"] == 0
    # the grade hooks: every configuration graded, saved and stopped by the thresholds
    grades = iter(np.linspace(0.5, 20.0, 100))
    out = al.fire(x0 + 0.3, inv_m, lambda x: -k * (x - x0), lambda x: next(grades), 1.0, 10.0, 1e-12, 100, 2.0, 10.0)
    g = np.linspace(0.5, 20.0, 100)
    first_break = int(np.argmax(g > 10.0))
    assert out["steps"] == first_break - 1 and len(out["gamma"]) == first_break + 1
    assert out["saved"] == [k for k in range(first_break) if g[k] > 2.0]


# -------------------------------------------------------------- maxvol -----
def test_maxvol_det_ratios_and_local_optimality_exhaustive():
    rng = np.random.default_rng(27)
    rows = rng.normal(size=(8, 3))
    A0 = rows[:3]
    cand = rows[3:]
    A, cand2, swaps = om.maxvol(A0, cand, threshold=1.0 + 1e-12)
    d = abs(np.linalg.det(A0))
    Acur, ccur = A0.copy(), cand.copy()
    for i, j, g in swaps:
        Acur[j], ccur[i] = ccur[i].copy(), Acur[j].copy()
        dn = abs(np.linalg.det(Acur))
        assert abs(dn / d - g) <= 1e-10 * g
        d = dn
    assert np.allclose(A, Acur)
    # no single swap increases |det A|
    for i in range(len(cand2)):
        for j in range(3):
            B = A.copy()
            B[j] = cand2[i]
            assert abs(np.linalg.det(B)) <= abs(np.linalg.det(A)) * (1 + 1e-9)
    # and the result is within the MaxVol bound of the exhaustive best
    best = max(abs(np.linalg.det(rows[list(s)])) for s in itertools.combinations(range(8), 3))
    assert abs(np.linalg.det(A)) >= best / 3 ** 1.5 - 1e-12


def test_sherman_morrison_matches_fresh_inverse():
    rng = np.random.default_rng(28)
    A = rng.normal(size=(6, 6))
    r = rng.normal(size=6)
    Ainv = np.linalg.inv(A)
    c = r @ Ainv
    j = int(np.argmax(np.abs(c)))
    e = np.zeros(6)
    e[j] = 1
    upd = Ainv - np.outer(Ainv[:, j], c - e) / c[j]
    A2 = A.copy()
    A2[j] = r
    assert np.allclose(upd, np.linalg.inv(A2), rtol=1e-12, atol=1e-12 * np.abs(upd).max())


# ----------------------------------------------------------- neighbors -----
@pytest.mark.parametrize("case", ["cubic", "triclinic_small", "slab"])
def test_neighbors_c_matches_python(case):
    rng = np.random.default_rng(29)
    if case == "cubic":
        pos, cell = _bcc((2, 2, 2))
        pbc = (1, 1, 1)
    elif case == "triclinic_small":
        cell = np.array([[3.1, 0, 0], [0.9, 2.9, 0], [0.4, -0.7, 3.3]])
        pos = rng.random((3, 3)) @ cell + rng.normal(0, 0.5, (3, 3))
        pbc = (1, 1, 1)
    else:
        cell = np.diag([6.0, 6.5, 20.0])
        pos = rng.random((10, 3)) @ cell
        pbc = (1, 1, 0)
    a = onb.neighbors(pos, cell, pbc, 5.0)
    b = onb.neighbors_py(pos, cell, pbc, 5.0)
    assert np.array_equal(np.c_[a.i, a.j, a.shift], np.c_[b.i, b.j, b.shift])
    # symmetry: (i, j, n) present iff (j, i, -n) present
    s = set(map(tuple, np.c_[a.i, a.j, a.shift]))
    assert all((j, i, -x, -y, -z) in s for i, j, x, y, z in s)


# ------------------------------------------------------------- fitting -----
def test_loss_gradient_matches_finite_differences():
    pot, theta, pos, types, cell = _setup(level=8, n_types=2, seed=30)
    pairs = _nbrs(pos, cell)
    rng = np.random.default_rng(31)
    cfgs = [(pos, types, cell, pairs)]
    tgt = [(rng.normal() * 10, rng.normal(size=pos.shape), rng.normal(size=(3, 3)))]
    L0, g = om.loss_and_grad(pot, theta, cfgs, tgt, 1.0, 0.01, 0.001)
    h = 1e-6
    for p in [0, 1, 4, pot.n_types + pot.n_lin + 3, pot.n_theta - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (om.loss_and_grad(pot, tp, cfgs, tgt, 1.0, 0.01, 0.001)[0]
              - om.loss_and_grad(pot, tm, cfgs, tgt, 1.0, 0.01, 0.001)[0]) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * np.abs(g).max(), (p, fd, g[p])
