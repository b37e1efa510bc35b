"""Autotuner of the P2P launch schedule: a thin wrapper of pmfmm_autotune.

Every work item writes its own partial sums and they are added in a fixed
order: the workgroup size and the grid leave the results bitwise alone, the
work-item size regroups the float64 sums (a change by rounding only).  The
schedule only decides how the uneven TaskGroup rows are cut into work items
(``chunk`` j leaves per item), how many wavefronts share a workgroup and its
LDS copy of the table (``wg_waves``), and how many persistent workgroups are
launched (``grid_wgs``, 0 = as many as fit).  The library times candidate
schedules on a built context with HIP events around the P2P kernel and
applies the fastest; results are cached in a text file keyed by device, pair
form and a coarse signature of the plan.
"""

from __future__ import annotations

import os

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pmfmm_tune.txt")


def candidates():
    """The library's default schedules: (chunk, wg_waves, grid_wgs)."""
    return [(chunk, wg, 0) for chunk in (0, 8, 16, 32, 64, 1 << 20) for wg in (2, 4, 8, 16)]


def autotune(ctx, out, stream=None, repeats: int = 3, cache_path: str = CACHE,
             use_cache: bool = True, cands=None, verbose: bool = False):
    """Pick the fastest schedule for the context's current plan.

    ``ctx`` is a built binding.Context, ``out`` a float64 CUDA tensor (n, 3)
    the forwards write into.  Returns (best schedule dict,
    {(chunk, wg_waves, grid_wgs): mean P2P ms}) (empty on a cache hit).
    """
    path = None
    if use_cache:
        path = cache_path
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    best, timed = ctx.autotune(out, stream, cands=cands, repeats=repeats, cache_path=path)
    results = {(r["chunk"], r["wg_waves"], r["grid_wgs"]): r["p2p_ms"] for r in timed
               if r["p2p_ms"] >= 0}
    if verbose:
        for k, v in sorted(results.items(), key=lambda kv: kv[1]):
            print(f"[tune] chunk {k[0]} wg {k[1]} grid {k[2]}: {v:.3f} ms", flush=True)
    return best, results
