"""ORB tree and the dual walk that yields the P2P and M2L task lists.

Test infrastructure (see the package docstring).  Float64 numpy.

Paper passages followed:
  * Sec. 2: an Orthogonal Recursive Bisection tree; the particles of a cell
    are shared equally between its two children until a cell holds at most
    MAXLEAF particles (a leaf).
  * Sec. 3: one traversal of the tree writes two task lists, M2L pairs and
    P2P pairs; a task <i, j> is the force on leaf (cell) i from leaf (cell) j.
  * Sec. 3.2: the task list is reordered by i (TaskGroup) and indexed by
    GroupIdx (start and length per i-leaf).
  * Sec. 2: the kernel is truncated at the cutoff radius.

Readings (the paper names the operations but not these details):
  * split axis: the axis of largest extent hi - lo of the cell's particles
    (first such axis on ties); the left child takes the floor(n/2) particles
    that are smallest by (coordinate on that axis, original index); a cell
    with n <= MAXLEAF is a leaf; inside a leaf particles are in ascending
    original index.  Cells are numbered in pre-order (parent, left subtree,
    right subtree), leaves in the order they are met; the particle order
    (``perm``) is the leaves' particles in leaf order.
  * per cell: lo / hi = exact min / max of its particles, centre
    c = 0.5 (lo + hi), half size hs = 0.5 (hi - lo), radius
    rad = sqrt((hs_x^2 + hs_y^2) + hs_z^2).  The centre is the expansion
    centre.
  * walk: start from (root, root, s) for all 27 image shifts s in {-1,0,1}^3
    (the shift moves the source by s L).  For a pair (t, u, s):
        R_a   = (c_u,a - c_t,a) + s_a L
        gap_a = max(|R_a| - (hs_t,a + hs_u,a), 0)    dmax_a = |R_a| + (hs_t,a + hs_u,a)
        gap2, dmax2, R2 = (v_x^2 + v_y^2) + v_z^2 of gap, dmax, R
      drop     if gap2 >= (r_cut * r_cut) * (1 + 2^-40);
      M2L      if the far field is on, dmax2 < (r_cut * r_cut) * (1 - 2^-40)
               and (rad_t + rad_u)^2 < (theta * theta) * R2;
      P2P      if both are leaves;
      else refine: split the cell of larger radius (a leaf is never split;
      equal radii split both).
    The guard factors make every rounding error fall on the safe side, so a
    particle pair inside the cutoff is never dropped and a pair sent to M2L
    lies wholly inside it; the per-pair cutoff of the P2P sum then decides.
  * the literal alternative (``centre_cut``): the kernel and its derivatives
    are cut at r_cut by the centre distance, so a pair passing the
    opening-angle test goes to M2L when R2 < r_cut * r_cut and is dropped
    otherwise, whatever part of it lies inside the cutoff.
    Every quantity is symmetric under (t, u, s) -> (u, t, -s), so the lists
    are symmetric.
  * canonical order: P2P tasks sorted by (i leaf, j leaf, shift code), M2L
    tasks by (target cell, source cell, shift code), with shift code
    (s_x + 1) + 3 (s_y + 1) + 9 (s_z + 1).

Every decision uses only correctly rounded float64 +, -, *, sqrt, abs, max
and comparisons in the order written above, so an independent builder that
follows the same text produces the same integers.

Parity: pinned by tests/test_oracle_tree.py (tree invariants, coverage of
every within-cutoff pair exactly once by P2P or by M2L against the brute-force
neighbour counts, list symmetry, empty M2L list for theta = 0; with the
centre cut, every within-cutoff pair covered exactly once by P2P, M2L or a
dropped accepted pair, each accepted pair on the right side of r_cut).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GUARD = 2.0 ** -40


def shift_vectors():
    """Shift code -> (s_x, s_y, s_z), code = (s_x+1) + 3 (s_y+1) + 9 (s_z+1)."""
    code = np.arange(27)
    return np.stack([code % 3 - 1, (code // 3) % 3 - 1, code // 9 - 1],
                    axis=1).astype(np.float64)


@dataclass
class Tree:
    perm: np.ndarray        # (N,) original index of each particle in leaf order
    lo: np.ndarray          # (C, 3)
    hi: np.ndarray          # (C, 3)
    first: np.ndarray       # (C,) first particle (leaf order)
    count: np.ndarray       # (C,)
    child: np.ndarray       # (C, 2) children, -1 for leaves
    parent: np.ndarray      # (C,) -1 for the root
    depth: np.ndarray       # (C,)
    leaf_of_cell: np.ndarray  # (C,) leaf id or -1
    leaf_cell: np.ndarray   # (n_leaves,) cell id of each leaf

    @property
    def centre(self):
        return 0.5 * (self.lo + self.hi)

    @property
    def half(self):
        return 0.5 * (self.hi - self.lo)

    @property
    def radius(self):
        h = self.half
        return np.sqrt((h[:, 0] * h[:, 0] + h[:, 1] * h[:, 1])
                       + h[:, 2] * h[:, 2])

    @property
    def n_leaves(self):
        return len(self.leaf_cell)

    @property
    def leaf_first(self):
        return self.first[self.leaf_cell]

    @property
    def leaf_count(self):
        return self.count[self.leaf_cell]


def build_orb(pos, max_leaf: int) -> Tree:
    """ORB tree of Sec. 2 with the readings of the module docstring."""
    pos = np.asarray(pos, np.float64)
    n = len(pos)
    if n < 1:
        raise ValueError("empty particle set")
    cells = []             # dicts in pre-order
    perm_parts = []
    leaf_cells = []
    cursor = [0]

    def rec(idx, parent, depth):
        sub = pos[idx]
        lo = sub.min(axis=0)
        hi = sub.max(axis=0)
        cid = len(cells)
        rec_ = dict(lo=lo, hi=hi, first=cursor[0], count=len(idx),
                    child=[-1, -1], parent=parent, depth=depth, leaf=-1)
        cells.append(rec_)
        if len(idx) <= max_leaf:
            rec_["leaf"] = len(leaf_cells)
            leaf_cells.append(cid)
            perm_parts.append(np.sort(idx))
            cursor[0] += len(idx)
            return cid
        ext = hi - lo
        axis = int(np.argmax(ext))            # first axis on ties
        order = np.lexsort((idx, sub[:, axis]))
        half = len(idx) // 2
        left = idx[order[:half]]
        right = idx[order[half:]]
        rec_["child"][0] = rec(left, cid, depth + 1)
        rec_["child"][1] = rec(right, cid, depth + 1)
        return cid

    rec(np.arange(n), -1, 0)
    return Tree(
        perm=np.concatenate(perm_parts),
        lo=np.array([c["lo"] for c in cells]),
        hi=np.array([c["hi"] for c in cells]),
        first=np.array([c["first"] for c in cells], np.int64),
        count=np.array([c["count"] for c in cells], np.int64),
        child=np.array([c["child"] for c in cells], np.int64),
        parent=np.array([c["parent"] for c in cells], np.int64),
        depth=np.array([c["depth"] for c in cells], np.int64),
        leaf_of_cell=np.array([c["leaf"] for c in cells], np.int64),
        leaf_cell=np.array(leaf_cells, np.int64),
    )


@dataclass
class Lists:
    p2p: np.ndarray         # (n_p2p, 3) int64: i leaf, j leaf, shift code
    m2l: np.ndarray         # (n_m2l, 3) int64: target cell, source cell, code
    p2p_row: np.ndarray     # (n_leaves + 1,) CSR start of each i-leaf
    m2l_row: np.ndarray     # (n_cells + 1,) CSR start of each target cell


def _sq3(v):
    return (v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]) + v[:, 2] * v[:, 2]


def dual_walk(tree: Tree, box: float, r_cut: float, theta: float,
              far_field: bool, centre_cut: bool = False,
              dropped: list | None = None) -> Lists:
    """Dual traversal of Sec. 3 with the readings of the module docstring.

    With ``dropped`` (a list) and ``centre_cut``, the accepted pairs the
    centre cut drops are appended to it as (t, u, s) rows."""
    c = tree.centre
    hs = tree.half
    rad = tree.radius
    leaf = tree.leaf_of_cell >= 0
    svec = shift_vectors() * box
    rc2 = r_cut * r_cut
    rc2_drop = rc2 * (1.0 + GUARD)
    rc2_m2l = rc2 * (1.0 - GUARD)
    th2 = theta * theta
    use_m2l = far_field and theta > 0.0

    t = np.zeros(27, np.int64)
    u = np.zeros(27, np.int64)
    s = np.arange(27, dtype=np.int64)
    p2p_out, m2l_out = [], []
    while t.size:
        R = (c[u] - c[t]) + svec[s]
        A = np.abs(R)
        H = hs[t] + hs[u]
        gap = np.maximum(A - H, 0.0)
        keep = _sq3(gap) < rc2_drop
        t, u, s, A, H, R = t[keep], u[keep], s[keep], A[keep], H[keep], R[keep]
        gone = np.zeros(t.size, bool)
        if use_m2l:
            dmax = A + H
            lhs = rad[t] + rad[u]
            mac = lhs * lhs < th2 * _sq3(R)
            if centre_cut:
                inside = _sq3(R) < rc2
                m2l = mac & inside
                gone = mac & ~inside
                if dropped is not None:
                    dropped.append(np.stack([t[gone], u[gone], s[gone]], axis=1))
            else:
                m2l = (_sq3(dmax) < rc2_m2l) & mac
        else:
            m2l = np.zeros(t.size, bool)
        m2l_out.append(np.stack([t[m2l], u[m2l], s[m2l]], axis=1))
        rest = ~m2l & ~gone
        t, u, s = t[rest], u[rest], s[rest]
        lt, lu = leaf[t], leaf[u]
        both = lt & lu
        p2p_out.append(np.stack([tree.leaf_of_cell[t[both]],
                                 tree.leaf_of_cell[u[both]], s[both]], axis=1))
        t, u, s, lt, lu = t[~both], u[~both], s[~both], lt[~both], lu[~both]
        rt, ru = rad[t], rad[u]
        split_t = ~lt & (lu | (rt > ru))
        split_u = ~lu & (lt | (ru > rt))
        split_b = ~lt & ~lu & (rt == ru)
        nt, nu, ns = [], [], []
        for k in (0, 1):
            nt.append(tree.child[t[split_t], k]); nu.append(u[split_t])
            ns.append(s[split_t])
            nt.append(t[split_u]); nu.append(tree.child[u[split_u], k])
            ns.append(s[split_u])
            for k2 in (0, 1):
                nt.append(tree.child[t[split_b], k])
                nu.append(tree.child[u[split_b], k2])
                ns.append(s[split_b])
        t = np.concatenate(nt)
        u = np.concatenate(nu)
        s = np.concatenate(ns)

    p2p = np.concatenate(p2p_out).astype(np.int64)
    m2l = np.concatenate(m2l_out).astype(np.int64)
    p2p = p2p[np.lexsort((p2p[:, 2], p2p[:, 1], p2p[:, 0]))]
    m2l = m2l[np.lexsort((m2l[:, 2], m2l[:, 1], m2l[:, 0]))]
    nl = tree.n_leaves
    nc = len(tree.lo)
    p2p_row = np.searchsorted(p2p[:, 0], np.arange(nl + 1))
    m2l_row = np.searchsorted(m2l[:, 0], np.arange(nc + 1))
    return Lists(p2p, m2l, p2p_row.astype(np.int64), m2l_row.astype(np.int64))


def candidate_pairs(tree: Tree, lists: Lists) -> int:
    """Particle pairs the P2P tasks evaluate (n_i * n_j summed over tasks).

    Pinned by tests/test_oracle_metrics.py: N^2 for an isolated cluster
    whose leaf pairs are all tasks, 9 for a hand-built two-leaf case, and
    32 * 32 per task for full leaves of 32."""
    npl = tree.leaf_count
    return int(np.sum(npl[lists.p2p[:, 0]] * npl[lists.p2p[:, 1]]))
