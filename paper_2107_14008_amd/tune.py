"""Autotuner of the P2P launch schedule (work-item size and workgroup shape).

The results of the P2P kernel do not depend on the schedule: every work item
writes its own partial sums and they are added in a fixed order.  The
schedule only decides how the uneven TaskGroup rows are cut into work items
(``chunk`` j leaves per item), how many wavefronts share a workgroup and its
LDS copy of the table (``wg_waves``), and how many persistent workgroups are
launched (``grid_wgs``, 0 = as many as fit).  ``autotune`` times candidate
schedules on a built context with the library's HIP-event timer and applies
the fastest; results are cached in a JSON file keyed by device, pair form and
a coarse signature of the workload.
"""

from __future__ import annotations

import json
import os
import time

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pmfmm_tune.json")


def _signature(lists: dict, params) -> str:
    n_items_bucket = int(round(2 * max(1.0, lists["n_p2p"]) ** 0.5)) // 64
    return "|".join(str(x) for x in (
        params.precision, params.trunc, params.table_size, params.table_level,
        lists["n_boxes"], lists["n_leaves"] // 1024, n_items_bucket))


def _device_name():
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


def candidates(n_cu: int = 256):
    """Schedules tried: (chunk, wg_waves, grid_wgs)."""
    out = []
    for chunk in (0, 8, 16, 32, 64, 1 << 20):
        for wg in (2, 4, 8, 16):
            out.append((chunk, wg, 0))
    return out


def autotune(ctx, out, stream=None, repeats: int = 3, cache_path: str = CACHE,
             use_cache: bool = True, cands=None, verbose: bool = False):
    """Pick the fastest schedule for the context's current plan.

    ``ctx`` is a binding.Context that has been built; ``out`` a float64 CUDA
    tensor (n, 3) the forward writes into.  Returns (best schedule dict,
    {schedule: mean P2P ms}).
    """
    import torch
    lists = ctx.lists()
    key = _device_name() + "|" + _signature(lists, ctx.params)
    cache = {}
    if use_cache and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    timing_before = ctx.params.timing
    if use_cache and key in cache:
        best = cache[key]
        ctx.set_eval(chunk=best["chunk"], wg_waves=best["wg_waves"],
                     grid_wgs=best["grid_wgs"], timing=timing_before)
        return best, {}
    results = {}
    for chunk, wg, grid in (cands or candidates()):
        ctx.set_eval(chunk=chunk, wg_waves=wg, grid_wgs=grid, timing=1)
        ctx.forward(out, stream)               # warm-up of this schedule
        ms = []
        for _ in range(repeats):
            ctx.forward(out, stream)
            ms.append(ctx.timings()["p2p_ms"])
        results[(chunk, wg, grid)] = sum(ms) / len(ms)
        if verbose:
            print(f"[tune] chunk {chunk} wg {wg} grid {grid}: "
                  f"{results[(chunk, wg, grid)]:.3f} ms", flush=True)
    torch.cuda.synchronize()
    (chunk, wg, grid), best_ms = min(results.items(), key=lambda kv: kv[1])
    best = dict(chunk=chunk, wg_waves=wg, grid_wgs=grid, p2p_ms=best_ms,
                when=time.time())
    ctx.set_eval(chunk=chunk, wg_waves=wg, grid_wgs=grid, timing=timing_before)
    if use_cache:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            json.dump(cache, open(cache_path, "w"), indent=1)
        except OSError:
            pass
    return best, results
