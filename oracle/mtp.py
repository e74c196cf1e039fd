"""Plain FP64 evaluation of the Moment Tensor Potential -- oracle side.

Test infrastructure only (see ``oracle/__init__.py``).  Everything is float64
PyTorch CPU code written straight from the definitions; derivatives are exact
(reverse- or forward-mode autograd of the plain definition), never
hand-derived, so that a mistake in a formula cannot be mirrored in its
derivative.

Parameter vector (paper Sec. II.B: theta = (xi_alpha, c^(beta)_{mu,z_i,z_j})):

    theta = [ xi_0 (N_types) | xi_1..xi_Nlin | c (N_rad, N_types, N_types, N_polyn) ]

Readings of passages the paper leaves open (each is also listed in the design
notes of the repository):

* eq. 2 has no constant term, yet the parameter counts 26 / 54 / 125 printed
  for levels 8 / 12 / 16 need exactly one more parameter per species: a
  per-species constant xi_0[z_i] is added to every site energy.
* T^(beta) in eq. 4 are "polynomial functions": read as Chebyshev polynomials
  of the first kind of degree beta-1 in x = (2r - R_min - R_cut)/(R_cut - R_min),
  not clamped for r < R_min.
* pairs with |r_ij| = R_cut are excluded (both f and f' vanish there).
* stress is S = -dE/d(eps) under x -> (I + eps) x applied to positions and
  cell vectors alike, in eV (not divided by the volume).
* grades use the full parameter vector minus N_rad(N_rad+1)/2 "gauge"
  columns (``gauge_columns``): the rows b_i are exactly rank deficient by
  that many directions (remixing f_mu with f_mu' for mu' <= mu is undone by
  xi), so the paper's m x m matrix A over all of theta is singular.  The
  LINEAR mode uses (onehot(z_i), B_alpha) only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg
import torch

from . import basis as _basis

F64 = torch.float64


# --------------------------------------------------------------------------
# model description
# --------------------------------------------------------------------------
@dataclass
class Potential:
    level: int
    n_types: int
    r_min: float
    r_cut: float
    n_polyn: int = 8

    def __post_init__(self):
        self.basis = _basis.basis(self.level)
        self.n_lin = len(self.basis)
        self.n_rad = _basis.n_rad(self.level)
        self.moments = _basis.moments_used(self.level)

    @property
    def n_c(self):
        return self.n_rad * self.n_types * self.n_types * self.n_polyn

    @property
    def n_theta(self):
        return self.n_types + self.n_lin + self.n_c

    def split(self, theta):
        """theta -> (xi0 [T], xi [N_lin], c [N_rad, T, T, N_polyn])."""
        T, L = self.n_types, self.n_lin
        return (theta[:T], theta[T:T + L],
                theta[T + L:].reshape(self.n_rad, T, T, self.n_polyn))


# --------------------------------------------------------------------------
# radial part, eq. 4
# --------------------------------------------------------------------------
def chebyshev(x, n):
    """T_0..T_{n-1}(x) by the three-term recurrence; shape x.shape + (n,)."""
    out = [torch.ones_like(x), x]
    while len(out) < n:
        out.append(2.0 * x * out[-1] - out[-2])
    return torch.stack(out[:n], dim=-1)


def radial_basis(pot: Potential, r):
    """Q_beta(r) = T^(beta)(r) (R_cut - r)^2, beta = 1..N_polyn (eq. 4)."""
    x = (2.0 * r - pot.r_min - pot.r_cut) / (pot.r_cut - pot.r_min)
    return chebyshev(x, pot.n_polyn) * ((pot.r_cut - r) ** 2).unsqueeze(-1)


def radial_functions(pot: Potential, c, r, zi, zj):
    """f_mu(|r|, z_i, z_j) = sum_beta c^(beta)_{mu,z_i,z_j} Q_beta(|r|); shape [P, N_rad]."""
    Q = radial_basis(pot, r)                      # [P, N_polyn]
    cij = c[:, zi, zj, :]                          # [N_rad, P, N_polyn]
    return torch.einsum("mpb,pb->pm", cij, Q)


# --------------------------------------------------------------------------
# moments (eq. 3), contractions and site energies (eq. 2)
# --------------------------------------------------------------------------
def moments(pot: Potential, c, rvec, i_idx, zi, zj, n_atoms):
    """Dense moment tensors M_{mu,nu}(n_i) = sum_j f_mu(|r_ij|) r_ij^{(x) nu} (eq. 3).

    rvec [P, 3] relative positions of all pairs, i_idx [P] owning atom.
    Returns {(mu, nu): tensor [n_atoms] + [3] * nu}.
    """
    r = torch.linalg.norm(rvec, dim=1)
    f = radial_functions(pot, c, r, zi, zj)       # [P, N_rad]
    out = {}
    for mu, nu in pot.moments:
        if nu == 0:
            term = f[:, mu]
        else:
            subs = ",".join(["p"] + [f"p{ch}" for ch in "abc"[:nu]])
            term = torch.einsum(subs + "->p" + "abc"[:nu], f[:, mu], *([rvec] * nu))
        acc = torch.zeros((n_atoms,) + (3,) * nu, dtype=F64)
        out[(mu, nu)] = acc.index_add(0, i_idx, term)
    return out


_LETTERS = "defghijklmnopqrstuvwxy"


def graph_value(g: _basis.Graph, M):
    """Full contraction of the moments of graph g: a sum over every labeling
    of its edges of the product of the tensor entries (Sec. II.A)."""
    idx = [[] for _ in range(g.n)]
    k = 0
    for p, q, mult in g.edge_list():
        for _ in range(mult):
            idx[p].append(_LETTERS[k])
            idx[q].append(_LETTERS[k])
            k += 1
    subs = ",".join("z" + "".join(s) for s in idx)
    return torch.einsum(subs + "->z", *[M[lab] for lab in g.labels])


def basis_values(pot: Potential, M):
    """B_alpha for every atom: products of connected graph values; [n, N_lin]."""
    gv = {g: graph_value(g, M) for g in _basis.connected_graphs(pot.level)}
    cols = []
    for bf in pot.basis:
        v = gv[bf.factors[0]]
        for g in bf.factors[1:]:
            v = v * gv[g]
        cols.append(v)
    return torch.stack(cols, dim=1)


def site_energies(pot: Potential, theta, rvec, i_idx, j_idx, types, n_atoms):
    """V(n_i) = xi_0[z_i] + sum_alpha xi_alpha B_alpha(n_i) (eq. 2, plus the
    species constant); returns (V [n_atoms], B [n_atoms, N_lin])."""
    xi0, xi, c = pot.split(theta)
    types_t = torch.as_tensor(types, dtype=torch.long)
    zi = types_t[i_idx]
    zj = types_t[j_idx]
    M = moments(pot, c, rvec, i_idx, zi, zj, n_atoms)
    B = basis_values(pot, M)
    return xi0[types_t] + B @ xi, B


# --------------------------------------------------------------------------
# systems
# --------------------------------------------------------------------------
@dataclass
class Pairs:
    """Neighborhood pairs (Sec. II.A): r_ij = x_j + shift . H - x_i."""
    i: np.ndarray       # [P] int64
    j: np.ndarray       # [P] int64
    shift: np.ndarray   # [P, 3] int64 (multiples of the cell vectors)


def _rvec(x, cell, pairs: Pairs):
    i = torch.as_tensor(pairs.i, dtype=torch.long)
    j = torch.as_tensor(pairs.j, dtype=torch.long)
    sh = torch.as_tensor(pairs.shift, dtype=F64)
    return x[j] + sh @ cell - x[i], i, j


def energy_forces_stress(pot: Potential, theta, pos, types, cell, pairs: Pairs):
    """Total energy (eq. 1), forces F = -dE/dx and stress S = -dE/deps.

    Returns (E float, F [N,3], S [3,3], V [N]) as NumPy float64.  E is the
    exactly rounded sum of the site energies (math.fsum).
    """
    n = len(pos)
    theta = torch.as_tensor(theta, dtype=F64)
    x = torch.tensor(pos, dtype=F64, requires_grad=True)
    eps = torch.zeros((3, 3), dtype=F64, requires_grad=True)
    D = torch.eye(3, dtype=F64) + eps
    xs = x @ D.T
    Hs = torch.as_tensor(cell, dtype=F64) @ D.T
    rvec, i, j = _rvec(xs, Hs, pairs)
    V, _ = site_energies(pot, theta, rvec, i, j, types, n)
    gx, geps = torch.autograd.grad(V.sum(), [x, eps])
    Vn = V.detach().numpy()
    return math.fsum(Vn.tolist()), -gx.numpy(), -geps.numpy(), Vn


def local_rvec(pos, cell, pairs: Pairs, atoms):
    """Pairs owned by the given atoms; owner = position of i within `atoms`."""
    loc = -np.ones(len(pos), dtype=np.int64)
    loc[np.asarray(atoms)] = np.arange(len(atoms))
    sel = loc[pairs.i] >= 0
    return Pairs(pairs.i[sel], pairs.j[sel], pairs.shift[sel]), loc[pairs.i[sel]]


def b_rows(pot: Potential, theta, pos, types, cell, pairs: Pairs, atoms=None, chunk=256):
    """b_i = dV(n_i)/dtheta over the full theta (Sec. II.D, eq. 10); [n_sel, |theta|].

    Computed by forward-mode differentiation of the plain site energy.
    """
    n = len(pos)
    atoms = np.arange(n) if atoms is None else np.asarray(atoms)
    theta = torch.as_tensor(theta, dtype=F64)
    x = torch.as_tensor(pos, dtype=F64)
    H = torch.as_tensor(cell, dtype=F64)
    types_np = np.asarray(types)
    out = []
    for s in range(0, len(atoms), chunk):
        sub = atoms[s:s + chunk]
        lp, owner = local_rvec(pos, cell, pairs, sub)
        rvec, _, j = _rvec(x, H, lp)
        own = torch.as_tensor(owner, dtype=torch.long)
        # types of the owners are those of the selected atoms
        t_local = types_np[sub]

        def fn(th):
            xi0, xi, c = pot.split(th)
            zi = torch.as_tensor(t_local, dtype=torch.long)[own]
            zj = torch.as_tensor(types_np, dtype=torch.long)[j]
            M = moments(pot, c, rvec, own, zi, zj, len(sub))
            B = basis_values(pot, M)
            return xi0[torch.as_tensor(t_local, dtype=torch.long)] + B @ xi

        out.append(torch.func.jacfwd(fn)(theta).detach().numpy())
    return np.concatenate(out, axis=0) if out else np.zeros((0, pot.n_theta))


def linear_rows(pot: Potential, theta, pos, types, cell, pairs: Pairs, atoms=None):
    """LINEAR-mode rows (onehot(z_i), B_alpha(n_i)); [n_sel, N_types + N_lin]."""
    n = len(pos)
    atoms = np.arange(n) if atoms is None else np.asarray(atoms)
    theta = torch.as_tensor(theta, dtype=F64)
    lp, owner = local_rvec(pos, cell, pairs, atoms)
    rvec, _, j = _rvec(torch.as_tensor(pos, dtype=F64), torch.as_tensor(cell, dtype=F64), lp)
    types_np = np.asarray(types)
    _, _, c = pot.split(theta)
    zi = torch.as_tensor(types_np[atoms], dtype=torch.long)[torch.as_tensor(owner)]
    zj = torch.as_tensor(types_np, dtype=torch.long)[j]
    M = moments(pot, c, rvec, torch.as_tensor(owner, dtype=torch.long), zi, zj, len(atoms))
    B = basis_values(pot, M).numpy()
    onehot = np.eye(pot.n_types)[types_np[atoms]]
    return np.concatenate([onehot, B], axis=1)


# --------------------------------------------------------------------------
# grades (Sec. II.C-D)
# --------------------------------------------------------------------------
def gauge_columns(pot: Potential, theta):
    """Columns of theta dropped in the FULL grade mode.

    For every mu, the null directions of the rows b_i move the block c_mu
    along c_0..c_mu; mu+1 columns of block c_mu are dropped, picked as the
    first mu+1 pivots of a column-pivoted QR of the (mu+1) x (T^2 N_polyn)
    matrix [c_0; ...; c_mu].  Returns sorted indices into theta.
    """
    _, _, c = pot.split(torch.as_tensor(theta, dtype=F64))
    c = c.numpy().reshape(pot.n_rad, -1)
    base = pot.n_types + pot.n_lin
    drop = []
    for mu in range(pot.n_rad):
        _, _, piv = scipy.linalg.qr(c[:mu + 1], mode="economic", pivoting=True)
        drop += [base + mu * c.shape[1] + int(p) for p in piv[:mu + 1]]
    return sorted(drop)


def kept_columns(pot: Potential, theta):
    drop = set(gauge_columns(pot, theta))
    return [k for k in range(pot.n_theta) if k not in drop]


def cfg_rows(rows, sizes):
    """Configuration-mode rows (Sec. II.C): b(cfg) = dE(cfg)/dtheta at the
    current theta.  With E = sum_i V_i (eq. 1) this is the sum of the
    neighborhood rows b_i over the configuration's atoms.  rows: [N, m] in
    configuration order; sizes: atoms per configuration.  Returns
    [n_cfg, m]."""
    rows = np.asarray(rows, dtype=np.float64)
    out = np.zeros((len(sizes), rows.shape[1]))
    o = 0
    for k, n in enumerate(sizes):
        out[k] = rows[o:o + int(n)].sum(axis=0)
        o += int(n)
    assert o == len(rows), "sizes do not add up to the number of rows"
    return out


def grades(rows, A):
    """gamma_i = max_p |c_ip| with c_i A = b_i solved by LU (Sec. II.D).

    Returns (gamma [n], argmax [n], C [n, m]); argmax takes the lowest index
    among ties.
    """
    lu = scipy.linalg.lu_factor(np.asarray(A, dtype=np.float64).T)
    C = scipy.linalg.lu_solve(lu, np.asarray(rows, dtype=np.float64).T).T
    absC = np.abs(C)
    return absC.max(axis=1), absC.argmax(axis=1), C


def maxvol(A, cand, threshold=1.001, max_swaps=None):
    """MaxVol swaps of candidate rows into the square matrix A (Sec. II.C).

    Repeatedly: C = cand A^-1; take the entry of largest |C_ij| (lowest i,
    then lowest j on ties); stop if it is <= threshold; else row j of A
    becomes candidate i (|det A| grows by |C_ij|) and the row it replaces
    takes the candidate's place in the pool.  Follows the plain definition:
    C is recomputed by a fresh solve after every swap.

    Returns (A_new, cand_new, swaps [(i, j, |C_ij|)]).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    cand = np.array(cand, dtype=np.float64, copy=True)
    m = A.shape[0]
    max_swaps = 10 * m if max_swaps is None else max_swaps
    swaps = []
    while len(swaps) < max_swaps and len(cand):
        _, _, C = grades(cand, A)
        flat = int(np.argmax(np.abs(C)))        # row-major: lowest i, then j
        i, j = divmod(flat, m)
        g = abs(C[i, j])
        if g <= threshold:
            break
        A[j], cand[i] = cand[i].copy(), A[j].copy()
        swaps.append((i, j, g))
    return A, cand, swaps


def initial_active_set(rows, m=None):
    """First m rows picked by a column-pivoted QR of rows^T (a greedy,
    rank-revealing choice of linearly independent rows); indices."""
    rows = np.asarray(rows, dtype=np.float64)
    m = rows.shape[1] if m is None else m
    _, _, piv = scipy.linalg.qr(rows.T, mode="economic", pivoting=True)
    return np.sort(piv[:m])


# --------------------------------------------------------------------------
# fitting objective (eq. 7) and its gradient
# --------------------------------------------------------------------------
def loss_and_grad(pot: Potential, theta, configs, targets, w_e, w_f, w_s):
    """L = sum_k [w_e (E_k-E_k^T)^2 + w_f sum_i |F_ik-F_ik^T|^2 + w_s sum_ab (S_abk-S^T_abk)^2]
    (eq. 7) and dL/dtheta by reverse-mode through the exact forces and stress.

    configs : list of (pos, types, cell, Pairs); targets : list of (E, F, S).
    """
    th = torch.tensor(theta, dtype=F64, requires_grad=True)
    total = torch.zeros((), dtype=F64)
    for (pos, types, cell, pairs), (Et, Ft, St) in zip(configs, targets):
        x = torch.tensor(pos, dtype=F64, requires_grad=True)
        eps = torch.zeros((3, 3), dtype=F64, requires_grad=True)
        D = torch.eye(3, dtype=F64) + eps
        rvec, i, j = _rvec(x @ D.T, torch.as_tensor(cell, dtype=F64) @ D.T, pairs)
        V, _ = site_energies(pot, th, rvec, i, j, types, len(pos))
        E = V.sum()
        gx, geps = torch.autograd.grad(E, [x, eps], create_graph=True)
        F, S = -gx, -geps
        total = total + w_e * (E - Et) ** 2 \
            + w_f * ((F - torch.as_tensor(Ft, dtype=F64)) ** 2).sum() \
            + w_s * ((S - torch.as_tensor(St, dtype=F64)) ** 2).sum()
    (g,) = torch.autograd.grad(total, [th])
    return float(total), g.numpy()
