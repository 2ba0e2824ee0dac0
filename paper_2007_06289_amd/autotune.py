"""Search for the fastest pass schedule of a plan (levels fused per HBM pass, column-tile width).

The transposed dyadic FHT runs log2 N butterfly levels (eq 19-21); each level performs the same
pairwise additions whichever pass executes it, so every schedule gives bit-identical images and
the search may demand exact equality with the default schedule.  The candidates are the
compositions of log2 N into at most ``max_passes`` parts; the library rejects the ones its
kernels cannot run (tile too large for LDS), each remaining one is timed on the caller's batch
with HIP events, and the fastest is applied to the plan and stored in a JSON cache keyed by
device, size, batch and filter shape.
"""
from __future__ import annotations

import json
import os

import torch

from . import api


def default_cache_path() -> str:
    return os.environ.get("FHTFBP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fhtfbp",
                                       "schedules.json"))


def cache_key(plan: api.Plan, batch: int) -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "") or props.name
    return (f"{arch}|cus={props.multi_processor_count}|n={plan.n}|batch={batch}|"
            f"order={plan.order}|groups={plan.groups}|flags={plan.flags}")


def compositions(total: int, max_parts: int, max_part: int):
    """Ordered ways of writing ``total`` as a sum of 1..max_parts parts, each in 1..max_part."""
    out = []

    def rec(rest, acc):
        if rest == 0:
            out.append(tuple(acc))
            return
        if len(acc) == max_parts:
            return
        for p in range(min(rest, max_part), 0, -1):
            rec(rest - p, acc + [p])

    rec(total, [])
    return out


def candidate_schedules(plan: api.Plan, max_passes: int | None = None,
                        widths=(7, 8, 9)) -> list[tuple[tuple[int, ...], int]]:
    """(levels, log2w) pairs to try; the plan's current schedule comes first.  By default no
    more passes than the current schedule (every extra pass moves the whole data set through
    HBM once more) and at most 6 levels in a column-tiled pass (the LDS limit)."""
    levels, log2w, first_max = plan.schedule()
    log2n = plan.n.bit_length() - 1
    if max_passes is None:
        max_passes = len(levels)
    cands = [(tuple(levels), log2w)]
    ws = [w for w in widths if w <= log2n] if log2n >= 8 else [log2w]
    for comp in compositions(log2n, max_passes, 6 if log2n >= 8 else log2n):
        if comp[0] > first_max:
            continue
        for w in ws:
            if (comp, w) not in cands:
                cands.append((comp, w))
    return cands


def _time(fn, reps: int) -> float:
    fn()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def tune(plan: api.Plan, lino: torch.Tensor, reps: int = 3, max_passes: int | None = None,
         cache_path: str | None = None, use_cache: bool = True, log=None) -> dict:
    """Time the candidate schedules of ``plan`` on ``lino`` ([B,4,N,N] on the GPU), apply the
    fastest and return {"levels", "log2w", "ms", "default_ms", "tried", "cached"}.  A result
    already in the cache is applied without timing when ``use_cache``."""
    B = int(lino.shape[0])
    path = cache_path or default_cache_path()
    key = cache_key(plan, B)
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if use_cache and key in cache:
        hit = cache[key]
        plan.set_schedule(hit["levels"], hit["log2w"])
        return dict(hit, cached=True)

    img = torch.empty((B, plan.n, plan.n), device=lino.device, dtype=torch.float32)
    ref = None
    best = None
    tried = 0
    default_ms = None
    for levels, w in candidate_schedules(plan, max_passes):
        try:
            plan.set_schedule(levels, w)
        except api.FbpError as e:
            if e.code in (api.FBP_ERANGE,):
                continue
            raise
        ms = _time(lambda: api.fbp_reconstruct(plan, lino, img), reps)
        tried += 1
        if ref is None:
            ref = img.clone()
            default_ms = ms
        elif not torch.equal(img, ref):
            raise RuntimeError(f"schedule {levels} w={w} changed the result")
        if log:
            log(f"schedule {list(levels)} log2w={w}: {ms:.3f} ms")
        if best is None or ms < best[0]:
            best = (ms, levels, w)
    ms, levels, w = best
    plan.set_schedule(levels, w)
    res = {"levels": list(levels), "log2w": int(w), "ms": round(ms, 4),
           "default_ms": round(default_ms, 4), "tried": tried}
    cache[key] = res
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return dict(res, cached=False)
