"""Brute-force short-range acceleration and its gradient (the definitions).

Test infrastructure (see the package docstring).  Float64 numpy.

What is computed (Sec. 2, Eq. (tr), with Alg. 2's dx = pos_j - pos_i):

    a_i = G sum_{j != i, 0 < |d_ij|^2 < r_cut^2} m_j T(|d_ij| / 2 r_s) d_ij / |d_ij|^3

where d_ij is the minimum-image displacement from particle i to particle j in
a periodic cube of side L.  The sharp cutoff is the paper's "numerically
truncate ... at cutoff radius" (Sec. 2).

Readings fixed here:
  * displacement: e = x_j - x_i per axis, then d = e + s L with the image
    shift s = -1 if e > L/2, +1 if e < -L/2, else 0 (each step one rounded
    float64 operation, in this order);
  * inclusion: 0 < r2 < r_cut^2 with r2 = (dx dx + dy dy) + dz dz evaluated
    without fused multiply-add, and r_cut^2 the rounded product r_cut * r_cut;
  * no softening (Alg. 2 has none); per-particle masses m_j in place of the
    single GM of Alg. 2.

Gradient of the loss L = sum_i w_i . a_i (not in the paper; derived from the
sum above).  With d = d_kl, r = |d|, g = T / r^3 and
h = g'(r) / r = -(3 T + (4 / sqrt(pi)) x^3 e^(-x^2)) / r^5, x = r / 2 r_s:

    dL/dx_k = G sum_{l in N(k)} [ m_k (g w_l + h (d.w_l) d) - m_l (g w_k + h (d.w_k) d) ]
    dL/dm_k = -G sum_{l in N(k)} g (w_l . d)

the delta function of the hard cutoff being left out (the gradient is the
almost-everywhere one).

Two independent evaluation routes are provided: ``all_pairs`` (every pair,
O(N^2), for small N) and ``brute_force`` (cell grid of side >= r_cut and its
27 neighbour cells).  Parity: pinned by tests/test_oracle_direct.py (route
agreement, the two-particle closed form, the perfect-lattice zero force,
translation invariance, momentum conservation, the Newtonian limit, and the
gradient against central finite differences).
"""

from __future__ import annotations

import math
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
from scipy.special import erfc

SQRT_PI = math.sqrt(math.pi)


def image_displacement(xi, xj, box):
    """d = (x_j - x_i) + s L with the minimum-image shift s in {-1, 0, 1}."""
    e = xj - xi
    s = np.zeros_like(e)
    s[e > 0.5 * box] = -1.0
    s[e < -0.5 * box] = 1.0
    return e + s * box


def _r2(d):
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def _T(x, table):
    """T(x) of Eq. (tr), or its Eq. (int) table form when ``table`` is
    (n_tab, level, rounding)."""
    if table is None:
        return erfc(x) + (2.0 / SQRT_PI) * x * np.exp(-x * x)
    from .truncation import T_table
    return T_table(x, table[0], table[1], table[2])


def _pair_accel(xi, xj, mj, box, r_s, rc2, table=None):
    """Acceleration on each row of xi from every row of xj (no G)."""
    d = image_displacement(xi[:, None, :], xj[None, :, :], box)
    r2 = _r2(d)
    ok = (r2 > 0.0) & (r2 < rc2)
    r2s = np.where(ok, r2, 1.0)
    r = np.sqrt(r2s)
    x = r / (2.0 * r_s)
    T = _T(x, table)
    g = np.where(ok, mj[None, :] * T / (r2s * r), 0.0)
    return np.einsum("ij,ijk->ik", g, d), ok.sum(axis=1)


def all_pairs(pos, mass, box, r_s, r_cut, G=1.0, targets=None, chunk=256,
              table=None):
    """O(N^2) minimum-image truncated sum; returns (acc, neighbour counts).

    ``table`` = (n_tab, level, rounding) replaces T by its Eq. (int) table.
    """
    pos = np.asarray(pos, np.float64)
    mass = np.asarray(mass, np.float64)
    rc2 = r_cut * r_cut
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    acc = np.zeros((len(idx), 3))
    cnt = np.zeros(len(idx), np.int64)
    for s in range(0, len(idx), chunk):
        sl = idx[s:s + chunk]
        a, c = _pair_accel(pos[sl], pos, mass, box, r_s, rc2, table)
        acc[s:s + chunk] = G * a
        cnt[s:s + chunk] = c
    return acc, cnt


# ---------------------------------------------------------------- cell grid

class CellGrid:
    """Cubic cell grid of side >= r_cut over the periodic box."""

    def __init__(self, pos, box, r_cut):
        self.box = box
        self.nc = max(1, int(math.floor(box / r_cut)))
        side = box / self.nc
        c = np.floor(pos / side).astype(np.int64)
        c = np.clip(c, 0, self.nc - 1)
        self.cell_of = (c[:, 0] * self.nc + c[:, 1]) * self.nc + c[:, 2]
        self.order = np.argsort(self.cell_of, kind="stable")
        counts = np.bincount(self.cell_of, minlength=self.nc ** 3)
        self.start = np.concatenate([[0], np.cumsum(counts)])

    def members(self, cid):
        return self.order[self.start[cid]:self.start[cid + 1]]

    def neighbours(self, cid):
        nc = self.nc
        cx, rem = divmod(cid, nc * nc)
        cy, cz = divmod(rem, nc)
        out = []
        for ox in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for oz in (-1, 0, 1):
                    out.append((((cx + ox) % nc) * nc + (cy + oy) % nc) * nc
                               + (cz + oz) % nc)
        return np.unique(np.asarray(out))


_WORK = {}
_PAIR_BLOCK = 1 << 21      # pairs evaluated per numpy block


def _init_worker(payload):
    _WORK.clear()
    _WORK.update(payload)


def _cells_job(cids):
    w = _WORK
    grid = w["grid"]
    fn = globals()[w["fn"]]
    out = []
    for cid in cids:
        ti = grid.members(cid)
        if w["mask"] is not None:
            ti = ti[w["mask"][ti]]
        if ti.size == 0:
            continue
        nb = np.concatenate([grid.members(c) for c in grid.neighbours(cid)])
        step = max(1, _PAIR_BLOCK // max(1, nb.size))
        for s in range(0, ti.size, step):
            out.append((ti[s:s + step], fn(ti[s:s + step], nb)))
    return out


def _start_method():
    """fork unless this process holds a GPU context (then fresh interpreters)."""
    import sys
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return "spawn"
    return "fork"


def _run_cells(pos, mass, box, r_cut, fn_name, targets, workers, extra=None):
    """Evaluate ``fn_name(targets_in_cell, neighbour_particles)`` per cell.

    Workers are forked, or started as fresh interpreters when this process
    has initialised a GPU, so that no device state is inherited.
    """
    grid = CellGrid(pos, box, r_cut)
    mask = None
    if targets is not None:
        mask = np.zeros(len(pos), bool)
        mask[np.asarray(targets)] = True
    payload = dict(pos=pos, mass=mass, grid=grid, mask=mask, fn=fn_name)
    if extra:
        payload.update(extra)
    cids = np.arange(grid.nc ** 3)
    if targets is not None:
        cids = np.unique(grid.cell_of[np.asarray(targets)])
    if workers is None:
        workers = min(len(os.sched_getaffinity(0)), 16)
    if workers <= 1 or len(cids) < 2:
        _init_worker(payload)
        return _cells_job(cids)
    parts = np.array_split(cids, min(len(cids), 4 * workers))
    results = []
    ctx = mp.get_context(_start_method())
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx,
                             initializer=_init_worker,
                             initargs=(payload,)) as ex:
        for r in ex.map(_cells_job, parts):
            results.extend(r)
    return results


def _force_fn(ti, nb):
    w = _WORK
    return _pair_accel(w["pos"][ti], w["pos"][nb], w["mass"][nb], w["box"],
                       w["r_s"], w["rc2"], w.get("table"))


def brute_force(pos, mass, box, r_s, r_cut, G=1.0, targets=None, workers=None,
                table=None):
    """Truncated minimum-image sum over a cell grid.

    Returns (acc, neighbour counts) for every particle, or for ``targets``
    (in the order given) when that is set.  ``workers`` processes share the
    target cells (default: the CPUs this process may run on, at most 16).
    ``table`` = (n_tab, level, rounding) replaces T by its Eq. (int) table.
    """
    pos = np.ascontiguousarray(pos, np.float64)
    mass = np.ascontiguousarray(mass, np.float64)
    if r_cut >= 0.5 * box:
        raise ValueError("r_cut must be below half the box")
    if math.floor(box / r_cut) < 3:
        return all_pairs(pos, mass, box, r_s, r_cut, G, targets, table=table)
    res = _run_cells(pos, mass, box, r_cut, "_force_fn", targets, workers,
                     dict(box=box, r_s=r_s, rc2=r_cut * r_cut, table=table))
    acc = np.zeros((len(pos), 3))
    cnt = np.zeros(len(pos), np.int64)
    for ti, (a, c) in res:
        acc[ti] = G * a
        cnt[ti] = c
    if targets is not None:
        t = np.asarray(targets)
        return acc[t], cnt[t]
    return acc, cnt


# ---------------------------------------------------------------- gradient

def _pair_grad(k_idx, l_idx):
    w = _WORK
    pos, mass, wv = w["pos"], w["mass"], w["w"]
    box, r_s, rc2 = w["box"], w["r_s"], w["rc2"]
    d = image_displacement(pos[k_idx][:, None, :], pos[l_idx][None, :, :], box)
    r2 = _r2(d)
    ok = (r2 > 0.0) & (r2 < rc2)
    r2s = np.where(ok, r2, 1.0)
    r = np.sqrt(r2s)
    x = r / (2.0 * r_s)
    ex = np.exp(-x * x)
    T = erfc(x) + (2.0 / SQRT_PI) * x * ex
    g = np.where(ok, T / (r2s * r), 0.0)
    h = np.where(ok, -(3.0 * T + (4.0 / SQRT_PI) * x ** 3 * ex)
                 / (r2s * r2s * r), 0.0)
    wk = wv[k_idx][:, None, :]
    wl = wv[l_idx][None, :, :]
    mk = mass[k_idx][:, None, None]
    ml = mass[l_idx][None, :, None]
    dwl = np.sum(d * wl, axis=-1)[..., None]
    dwk = np.sum(d * wk, axis=-1)[..., None]
    gg = g[..., None]
    hh = h[..., None]
    ta = mk * (gg * wl + hh * dwl * d)
    tb = ml * (gg * wk + hh * dwk * d)
    gm = -(g * dwl[..., 0])
    # sums of term magnitudes: the scale a rounding error is measured against
    sx = (np.linalg.norm(ta, axis=-1) + np.linalg.norm(tb, axis=-1)).sum(axis=1)
    sm = np.abs(gm).sum(axis=1)
    return (ta - tb).sum(axis=1), gm.sum(axis=1), sx, sm


def gradient(pos, mass, w, box, r_s, r_cut, G=1.0, targets=None, workers=None,
             with_scale=False):
    """dL/dpos (N, 3) and dL/dmass (N) of L = sum_i w_i . a_i.

    With ``with_scale`` also the per-particle sums of the magnitudes of the
    summed pair terms (for dL/dpos and dL/dmass): a sum with heavy
    cancellation is only resolved to rounding times this scale.
    """
    pos = np.ascontiguousarray(pos, np.float64)
    mass = np.ascontiguousarray(mass, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    extra = dict(box=box, r_s=r_s, rc2=r_cut * r_cut, w=w)
    if math.floor(box / r_cut) < 3:
        _init_worker(dict(pos=pos, mass=mass, **extra))
        idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
        gx, gm, sx, sm = _pair_grad(idx, np.arange(len(pos)))
        if with_scale:
            return G * gx, G * gm, abs(G) * sx, abs(G) * sm
        return G * gx, G * gm
    res = _run_cells(pos, mass, box, r_cut, "_pair_grad", targets, workers,
                     extra)
    gx = np.zeros((len(pos), 3))
    gm = np.zeros(len(pos))
    sx = np.zeros(len(pos))
    sm = np.zeros(len(pos))
    for ti, (a, b, c, e) in res:
        gx[ti] = G * a
        gm[ti] = G * b
        sx[ti] = abs(G) * c
        sm[ti] = abs(G) * e
    if targets is not None:
        t = np.asarray(targets)
        gx, gm, sx, sm = gx[t], gm[t], sx[t], sm[t]
    if with_scale:
        return gx, gm, sx, sm
    return gx, gm


def loss(pos, mass, w, box, r_s, r_cut, G=1.0, workers=None):
    """L = sum_i w_i . a_i with the brute-force accelerations."""
    acc, _ = brute_force(pos, mass, box, r_s, r_cut, G, workers=workers)
    return float(np.sum(w * acc))
