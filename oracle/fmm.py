"""Truncated FMM of Sec. 2 on the oracle's own tree and task lists.

Test infrastructure (see the package docstring).  Float64 numpy.

Paper passages followed (Sec. 2): P2M (particles of a leaf to its
multipole), M2M (children to parent, the pass-up), M2L (the equation
L_n(z_B) = sum_{|m| <= p - |n|} M_m(z_A) D_{n+m}(z_B - z_A)), L2L (parent
local to child local), L2P (local expansion to particle force) and P2P
(direct pairs of neighbouring leaves); the P2P and M2L task lists of Sec. 3.

Expansion convention (a reading; the paper refers elsewhere for it).  For a
source cell A with centre z_A and a target cell B with centre z_B, and the
image shift s of the source, write R = z_B - (z_A + s L),
x = z_B + u (target) and y = z_A + s L + v (source).  Taylor expansion of the
kernel psi(x - y) = psi(R + u - v) gives

  M_m(z_A) = sum_j m_j (z_A - y_j)^m / m!                      (P2M)
  M_m(z_P) = sum_{k <= m} M_k(z_C) (z_P - z_C)^(m-k) / (m-k)!  (M2M)
  L_n(z_B) = sum_{|m| <= p-|n|} M_m(z_A) D_{n+m}(R)            (M2L)
  L_n(z_c) = sum_{k >= n, |k| <= p} L_k(z_P) (z_c - z_P)^(k-n) / (k-n)!  (L2L)
  a(x)     = G grad_u sum_n L_n u^n / n!,  u = x - z_B          (L2P)

with D_k = d^k psi the full Cartesian derivative tensor (``truncation``),
multi-index powers and factorials taken per axis, and all of M, L, D of
total order <= p.  The acceleration sign follows from
a(x) = G grad_x sum_j m_j psi(|x - y_j|) for the attractive kernel.

P2P pairs use the task's shift: d = (x_j - x_i) + s L, included when
0 < r2 < r_cut^2 as in ``direct``.

Adjoint (``fmm_gradient``; not in the paper): the gradient of
L = sum_i w_i . a_i through the P2P pairs of the task lists and through the
far-field operators, each transposed and applied in reverse order (L2P^T,
L2L^T children to parents, M2L^T, M2M^T parents to children, P2M^T), with
the tree, the lists and the expansion centres held fixed.

Parity: pinned by tests/test_oracle_fmm.py (P2M/M2M and L2L against direct
expansion about the new centre, M2L + L2P against the direct sum for
separated clusters with error falling as p grows, theta = 0 reducing to the
brute-force sum, and FMM-vs-brute-force error on clustered inputs; the
adjoint against central differences of the far-field force, against the
brute-force gradient at theta = 0, and converging to it as p grows).
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import truncation as tr
from .tree import Lists, Tree, build_orb, dual_walk, shift_vectors

SQRT_PI = math.sqrt(math.pi)


def _powers(v, k):
    """prod_a v_a^k_a / k_a! for rows of v."""
    out = np.ones(len(v))
    for a in range(3):
        out = out * v[:, a] ** k[a] / math.factorial(k[a])
    return out


def p2m(tree: Tree, pos, mass, p):
    """Multipoles of every leaf about its centre: dict index -> (C,) array."""
    mi = tr.multi_indices(p)
    nc = len(tree.lo)
    M = {k: np.zeros(nc) for k in mi}
    c = tree.centre
    for leaf, cell in enumerate(tree.leaf_cell):
        f, n = tree.first[cell], tree.count[cell]
        idx = tree.perm[f:f + n]
        v = c[cell][None, :] - pos[idx]
        for k in mi:
            M[k][cell] = float(np.sum(mass[idx] * _powers(v, k)))
    return M


def m2m(tree: Tree, M, p):
    """Pass-up: internal cells from their children, deepest cells first."""
    mi = tr.multi_indices(p)
    c = tree.centre
    for cell in range(len(tree.lo) - 1, -1, -1):
        if tree.leaf_of_cell[cell] >= 0:
            continue
        for ch in tree.child[cell]:
            dz = (c[cell] - c[ch])[None, :]
            for m in mi:
                acc = 0.0
                for k in mi:
                    if all(k[a] <= m[a] for a in range(3)):
                        mk = (m[0] - k[0], m[1] - k[1], m[2] - k[2])
                        acc += M[k][ch] * float(_powers(dz, mk)[0])
                M[m][cell] += acc
    return M


def m2l(tree: Tree, lists: Lists, M, p, box, r_s):
    """Local expansions from the M2L task list."""
    mi = tr.multi_indices(p)
    nc = len(tree.lo)
    L = {k: np.zeros(nc) for k in mi}
    if len(lists.m2l) == 0:
        return L
    c = tree.centre
    t, u, s = lists.m2l[:, 0], lists.m2l[:, 1], lists.m2l[:, 2]
    R = c[t] - (c[u] + shift_vectors()[s] * box)
    D = tr.derivative_tensor(R, p, r_s)
    for n in mi:
        acc = np.zeros(len(t))
        for m in mi:
            if sum(n) + sum(m) <= p:
                nm = (n[0] + m[0], n[1] + m[1], n[2] + m[2])
                acc = acc + M[m][u] * D[nm]
        np.add.at(L[n], t, acc)
    return L


def l2l(tree: Tree, L, p):
    """Pass-down: every child adds its parent's shifted expansion (pre-order)."""
    mi = tr.multi_indices(p)
    c = tree.centre
    for cell in range(1, len(tree.lo)):
        par = tree.parent[cell]
        dz = (c[cell] - c[par])[None, :]
        for n in mi:
            acc = 0.0
            for k in mi:
                if sum(k) <= p and all(k[a] >= n[a] for a in range(3)):
                    kn = (k[0] - n[0], k[1] - n[1], k[2] - n[2])
                    acc += L[k][par] * float(_powers(dz, kn)[0])
            L[n][cell] += acc
    return L


def l2p(tree: Tree, L, pos, p):
    """Gradient of each leaf's local polynomial at its particles (no G)."""
    mi = tr.multi_indices(p)
    acc = np.zeros((len(pos), 3))
    c = tree.centre
    for cell in tree.leaf_cell:
        f, n = tree.first[cell], tree.count[cell]
        idx = tree.perm[f:f + n]
        u = pos[idx] - c[cell][None, :]
        for nidx in mi:
            coef = L[nidx][cell]
            if coef == 0.0:
                continue
            for a in range(3):
                if nidx[a] >= 1:
                    km = list(nidx)
                    km[a] -= 1
                    acc[idx, a] += coef * _powers(u, tuple(km))
    return acc


def p2p(tree: Tree, lists: Lists, pos, mass, box, r_s, r_cut):
    """Direct pairs of every P2P task with its shift (no G)."""
    acc = np.zeros((len(pos), 3))
    rc2 = r_cut * r_cut
    sv = shift_vectors() * box
    lf, lc = tree.leaf_first, tree.leaf_count
    for i in range(tree.n_leaves):
        a0, a1 = lists.p2p_row[i], lists.p2p_row[i + 1]
        if a0 == a1:
            continue
        ti = tree.perm[lf[i]:lf[i] + lc[i]]
        src, shf = [], []
        for j, s in lists.p2p[a0:a1, 1:]:
            src.append(tree.perm[lf[j]:lf[j] + lc[j]])
            shf.append(np.repeat(s, lc[j]))
        src = np.concatenate(src)
        shf = np.concatenate(shf)
        d = (pos[src][None, :, :] - pos[ti][:, None, :]) + sv[shf][None, :, :]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        ok = (r2 > 0.0) & (r2 < rc2)
        r2s = np.where(ok, r2, 1.0)
        r = np.sqrt(r2s)
        x = r / (2.0 * r_s)
        T = erfc(x) + (2.0 / SQRT_PI) * x * np.exp(-x * x)
        g = np.where(ok, mass[src][None, :] * T / (r2s * r), 0.0)
        acc[ti] += np.einsum("ij,ijk->ik", g, d)
    return acc


# ---- Adjoint (not in the paper): the gradient of L = sum_i w_i . a_i through
# the same operators, each replaced by its transpose and applied in reverse
# order, with the tree, the task lists and the expansion centres held fixed
# (the centres are the cells' bounding-box centres; the gradient leaves out
# their dependence on the extreme particles of each cell).

def _e(k, a, sign):
    kk = list(k)
    kk[a] += sign
    return tuple(kk)


def l2p_transpose(tree: Tree, w, pos, p):
    """dL/dL_n(B) = sum_{i in B} w_i . grad_u [u^n / n!] at u = x_i - z_B
    for every leaf B (the transpose of L2P, no G)."""
    mi = tr.multi_indices(p)
    nc = len(tree.lo)
    Lb = {k: np.zeros(nc) for k in mi}
    c = tree.centre
    for cell in tree.leaf_cell:
        f, n = tree.first[cell], tree.count[cell]
        idx = tree.perm[f:f + n]
        u = pos[idx] - c[cell][None, :]
        for k in mi:
            tot = 0.0
            for a in range(3):
                if k[a] >= 1:
                    tot += float(np.sum(w[idx, a] * _powers(u, _e(k, a, -1))))
            Lb[k][cell] = tot
    return Lb


def l2l_transpose(tree: Tree, Lb, p):
    """Transpose of the pass-down: each cell adds its children's adjoints,
    shifted back, deepest cells first (reverse pre-order)."""
    mi = tr.multi_indices(p)
    c = tree.centre
    for cell in range(len(tree.lo) - 1, 0, -1):
        par = tree.parent[cell]
        dz = (c[cell] - c[par])[None, :]
        for k in mi:
            acc = 0.0
            for n in mi:
                if all(n[a] <= k[a] for a in range(3)):
                    kn = (k[0] - n[0], k[1] - n[1], k[2] - n[2])
                    acc += Lb[n][cell] * float(_powers(dz, kn)[0])
            Lb[k][par] += acc
    return Lb


def m2l_transpose(tree: Tree, lists: Lists, Lb, p, box, r_s):
    """dL/dM_m(A) = sum over tasks (B, A, s) of sum_n dL/dL_n(B) D_{n+m}(R),
    R = z_B - (z_A + s L): the M2L equation read from L back to M."""
    mi = tr.multi_indices(p)
    nc = len(tree.lo)
    Mb = {k: np.zeros(nc) for k in mi}
    if len(lists.m2l) == 0:
        return Mb
    c = tree.centre
    t, u, s = lists.m2l[:, 0], lists.m2l[:, 1], lists.m2l[:, 2]
    R = c[t] - (c[u] + shift_vectors()[s] * box)
    D = tr.derivative_tensor(R, p, r_s)
    for m in mi:
        acc = np.zeros(len(t))
        for n in mi:
            if sum(n) + sum(m) <= p:
                nm = (n[0] + m[0], n[1] + m[1], n[2] + m[2])
                acc = acc + Lb[n][t] * D[nm]
        np.add.at(Mb[m], u, acc)
    return Mb


def m2m_transpose(tree: Tree, Mb, p):
    """Transpose of the pass-up: each child adds its parent's adjoint,
    parents first (pre-order)."""
    mi = tr.multi_indices(p)
    c = tree.centre
    for cell in range(len(tree.lo)):
        if tree.leaf_of_cell[cell] >= 0:
            continue
        for ch in tree.child[cell]:
            dz = (c[cell] - c[ch])[None, :]
            for k in mi:
                acc = 0.0
                for m in mi:
                    if all(k[a] <= m[a] for a in range(3)):
                        mk = (m[0] - k[0], m[1] - k[1], m[2] - k[2])
                        acc += Mb[m][cell] * float(_powers(dz, mk)[0])
                Mb[k][ch] += acc
    return Mb


def far_gradient(tree: Tree, lists: Lists, pos, mass, w, box, r_s, p):
    """dL/dpos (N, 3) and dL/dmass (N) of the far-field part (no G).

    Particle k in leaf A, u = x_k - z_A, v = z_A - x_k:
      from L2P:  Hess phi_A(u) w_k, phi_A(u) = sum_n L_n(A) u^n / n!
      from P2M:  m_k d/dx_k sum_m Mb_m(A) v^m / m!  and  sum_m Mb_m(A) v^m / m!
    with Mb = dL/dM of the leaf multipoles."""
    mi = tr.multi_indices(p)
    M = m2m(tree, p2m(tree, pos, mass, p), p)
    L = l2l(tree, m2l(tree, lists, M, p, box, r_s), p)
    Lb = l2l_transpose(tree, l2p_transpose(tree, w, pos, p), p)
    Mb = m2m_transpose(tree, m2l_transpose(tree, lists, Lb, p, box, r_s), p)
    gx = np.zeros((len(pos), 3))
    gm = np.zeros(len(pos))
    c = tree.centre
    for cell in tree.leaf_cell:
        f, n = tree.first[cell], tree.count[cell]
        idx = tree.perm[f:f + n]
        u = pos[idx] - c[cell][None, :]
        v = -u
        for k in mi:
            gm[idx] += Mb[k][cell] * _powers(v, k)
            for a in range(3):
                if k[a] >= 1:
                    gx[idx, a] -= mass[idx] * Mb[k][cell] * _powers(v, _e(k, a, -1))
                for b in range(3):
                    if k[a] >= 1 and _e(k, a, -1)[b] >= 1:
                        kab = _e(_e(k, a, -1), b, -1)
                        gx[idx, a] += L[k][cell] * _powers(u, kab) * w[idx, b]
    return gx, gm


def p2p_gradient(tree: Tree, lists: Lists, pos, mass, w, box, r_s, r_cut):
    """dL/dpos and dL/dmass of the P2P part over the task lists (no G):
    the transpose of ``p2p``, gathered over each particle's own rows (the
    lists are symmetric).  With d = x_l + s L - x_k, g = T / r^3 and
    h = g'(r) / r:
      dL/dx_k = m_k sum_l (g w_l + h (d.w_l) d) - sum_l m_l (g w_k + h (d.w_k) d)
      dL/dm_k = -sum_l g (w_l . d)."""
    gx = np.zeros((len(pos), 3))
    gm = np.zeros(len(pos))
    rc2 = r_cut * r_cut
    sv = shift_vectors() * box
    lf, lc = tree.leaf_first, tree.leaf_count
    for i in range(tree.n_leaves):
        a0, a1 = lists.p2p_row[i], lists.p2p_row[i + 1]
        if a0 == a1:
            continue
        tk = tree.perm[lf[i]:lf[i] + lc[i]]
        src, shf = [], []
        for j, s in lists.p2p[a0:a1, 1:]:
            src.append(tree.perm[lf[j]:lf[j] + lc[j]])
            shf.append(np.repeat(s, lc[j]))
        src = np.concatenate(src)
        shf = np.concatenate(shf)
        d = (pos[src][None, :, :] - pos[tk][:, None, :]) + sv[shf][None, :, :]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        ok = (r2 > 0.0) & (r2 < rc2)
        r2s = np.where(ok, r2, 1.0)
        r = np.sqrt(r2s)
        x = r / (2.0 * r_s)
        ex = np.exp(-x * x)
        T = erfc(x) + (2.0 / SQRT_PI) * x * ex
        g = np.where(ok, T / (r2s * r), 0.0)
        h = np.where(ok, -(3.0 * T + (4.0 / SQRT_PI) * x ** 3 * ex) / (r2s * r2s * r), 0.0)
        wl = w[src][None, :, :]
        wk = w[tk][:, None, :]
        dwl = np.sum(d * wl, -1)
        dwk = np.sum(d * wk, -1)
        A = np.sum(g[..., None] * wl + (h * dwl)[..., None] * d, 1)
        Bv = np.sum((mass[src][None, :] * g)[..., None] * wk
                    + (mass[src][None, :] * h * dwk)[..., None] * d, 1)
        gx[tk] += mass[tk][:, None] * A - Bv
        gm[tk] += -np.sum(g * dwl, 1)
    return gx, gm


def fmm_gradient(pos, mass, w, box, r_s, r_cut, max_leaf, order, theta, G=1.0,
                 tree=None, lists=None, return_parts=False, centre_cut=False):
    """dL/dpos (N, 3) and dL/dmass (N) of L = sum_i w_i . a_i for the
    accelerations of ``fmm_forces`` (input order), tree, lists and
    expansion centres held fixed."""
    pos = np.asarray(pos, np.float64)
    mass = np.asarray(mass, np.float64)
    w = np.asarray(w, np.float64)
    far = order >= 0 and theta > 0.0
    if tree is None:
        tree = build_orb(pos, max_leaf)
    if lists is None:
        lists = dual_walk(tree, box, r_cut, theta, far, centre_cut)
    nx, nm = p2p_gradient(tree, lists, pos, mass, w, box, r_s, r_cut)
    fx, fm = np.zeros_like(nx), np.zeros_like(nm)
    if far and len(lists.m2l):
        fx, fm = far_gradient(tree, lists, pos, mass, w, box, r_s, order)
    if return_parts:
        return G * (nx + fx), G * (nm + fm), G * fx, G * fm, tree, lists
    return G * (nx + fx), G * (nm + fm)


def fmm_forces(pos, mass, box, r_s, r_cut, max_leaf, order, theta, G=1.0,
               tree=None, lists=None, return_parts=False, centre_cut=False):
    """Short-range accelerations by the truncated FMM (input order).

    order < 0 or theta <= 0 gives the plain P2P sum over the task lists;
    ``centre_cut`` selects the literal reading of the truncation for M2L
    (``tree.dual_walk``).
    """
    pos = np.asarray(pos, np.float64)
    mass = np.asarray(mass, np.float64)
    far = order >= 0 and theta > 0.0
    if tree is None:
        tree = build_orb(pos, max_leaf)
    if lists is None:
        lists = dual_walk(tree, box, r_cut, theta, far, centre_cut)
    near = p2p(tree, lists, pos, mass, box, r_s, r_cut)
    farf = np.zeros_like(near)
    if far and len(lists.m2l):
        M = p2m(tree, pos, mass, order)
        M = m2m(tree, M, order)
        L = m2l(tree, lists, M, order, box, r_s)
        L = l2l(tree, L, order)
        farf = l2p(tree, L, pos, order)
    acc = G * (near + farf)
    if return_parts:
        return acc, G * near, G * farf, tree, lists
    return acc
