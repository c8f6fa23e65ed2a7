"""Autotuner of the library's launch shapes.

What it searches, per plane class (operator type, N, kernel width w,
transfer function, log2 of the point count):
  * spread_chunk      -- records per spreading workgroup (1792 or the small size),
  * interp_chunk      -- records per interpolation workgroup (1024 .. 8192),
  * bin_range_points  -- points per binning workgroup (automatic or 4096 .. 65535),
  * spread_method     -- spreading on the matrix cores or by register gather,
  * bin_tile          -- bin side, 32 or 64 fine cells (64: fewer duplicated
                         records and bins, larger workgroups),
and, per batch, the graph form (grouped stage launches or per-plane branches)
and the number of parallel branches of the per-plane form (1 .. 4).

Each candidate is timed on the GPU with HIP events as the one-shot operation
it tunes (set_points + execute for a plane, a whole graph replay for a
batch), median of a few repetitions, by coordinate descent from the defaults.
Results are cached in a JSON file (NUASM_TUNE_CACHE, else
~/.cache/nuasm/tune.json) keyed by the plane class, so later plans and
batches of the same shapes reuse them without timing anything.
"""
from __future__ import annotations

import json
import math
import os
import statistics

import torch

from . import FORWARD_ONLY, Batch, NuasmError, Plan, make_params

CANDIDATES = {
    "bin_range_points": (0, 2048, 4096, 16384, 65535),
    "interp_chunk": (0, 1024, 4096, 8192),
    "spread_chunk": (0, 896),
    "spread_method": (0, 1),
    "bin_tile": (0, 64),
}
DEFAULT = {"spread_chunk": 0, "interp_chunk": 0, "bin_range_points": 0, "spread_method": 0, "bin_tile": 0}


def cache_path() -> str:
    return os.environ.get("NUASM_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "nuasm",
                                                              "tune.json")


class TuneCache:
    """JSON cache {key: tuning dict}."""

    def __init__(self, path: str | None = None):
        self.path = path or cache_path()
        self.data = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def plane_key(spec: dict, M: int) -> str:
    """Plane class of a make_params spec with M points."""
    p = make_params(**spec)
    w = max(2, min(16, int(math.ceil(-math.log10(p.tol) - 1e-9)) + 1))
    mb = int(round(math.log2(max(M, 1))))
    tf = "fresnel" if p.tf == 1 else "asm"
    fwd = ":fwd" if p.flags & FORWARD_ONLY else ""  # one record per point
    return f"plane:t{p.type}:N{p.N}:w{w}:{tf}:m{mb}{fwd}"


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return statistics.median(out)


def tune_plane(spec: dict, x: torch.Tensor, y: torch.Tensor, inp: torch.Tensor, reps: int = 3) -> dict:
    """Coordinate descent over CANDIDATES for one plane (binned points);
    returns the best tuning and its one-shot time in ms."""
    plan = Plan(**{**spec, "defer_range_check": True})

    def run(t):
        try:
            plan.set_tuning(**t)
        except NuasmError:
            return float("inf")  # a combination the library does not take

        def once():
            plan.set_points(x, y)
            return plan.execute(inp)
        return _time(once, reps)

    best = dict(DEFAULT)
    best_ms = run(best)
    # two sweeps of coordinate descent: a setting can pay only once another
    # has changed (a 64 x 64 bin tile wants other chunk sizes)
    for _ in range(2):
        changed = False
        for name, cands in CANDIDATES.items():
            for v in cands:
                if v == best[name]:
                    continue
                t = dict(best)
                t[name] = v
                ms = run(t)
                if ms < best_ms * 0.98:  # keep the simpler setting unless clearly faster
                    best, best_ms, changed = t, ms, True
        if not changed:
            break
    plan.check_points()
    return {**best, "ms": best_ms}


def tune_batch(batch: Batch, specs, xs, ys, ins, outs, cache: TuneCache | None = None, reps: int = 3) -> dict:
    """Tune every plane class of a batch (cached classes are reused), apply
    the tunings to the batch's planes, then pick the number of graph branches
    by timing whole graph runs.  Returns a summary."""
    cache = cache if cache is not None else TuneCache()
    tuned, reused = 0, 0
    for p, spec in enumerate(specs):
        key = plane_key(spec, xs[p].numel())
        t = cache.get(key)
        if t is None:
            t = tune_plane(spec, xs[p], ys[p], ins[p], reps)
            cache.put(key, t)
            tuned += 1
        else:
            reused += 1
        batch.set_tuning(p, **{k: t.get(k, 0) for k in DEFAULT})
    bkey = "batch:" + ",".join(sorted({plane_key(s, xs[p].numel()) for p, s in enumerate(specs)}))
    choice = cache.get(bkey)
    times = {}
    if choice is None or "grouped" not in choice:
        # graph forms: grouped stage launches, or per-plane launches on 1..4 branches
        batch.set_grouped(True)
        times["grouped"] = _time(lambda: batch.run(xs, ys, ins, outs), reps)
        batch.set_grouped(False)
        for k in range(1, min(4, len(specs)) + 1):
            batch.set_branches(k)
            times[str(k)] = _time(lambda: batch.run(xs, ys, ins, outs), reps)
        best = min(times, key=times.get)
        choice = {"grouped": best == "grouped", "branches": 1 if best == "grouped" else int(best),
                  "ms": times[best]}
        cache.put(bkey, choice)
    batch.set_grouped(bool(choice["grouped"]))
    if not choice["grouped"]:
        batch.set_branches(int(choice["branches"]))
    cache.save()
    return {"planes_tuned": tuned, "planes_from_cache": reused, "grouped": bool(choice["grouped"]),
            "branches": int(choice["branches"]), "form_ms": times, "cache": cache.path}


def apply_cached(batch: Batch, specs, Ms, cache: TuneCache | None = None) -> int:
    """Apply cached tunings to a batch's planes without timing anything;
    returns how many planes had one."""
    cache = cache if cache is not None else TuneCache()
    n = 0
    for p, spec in enumerate(specs):
        t = cache.get(plane_key(spec, int(Ms[p])))
        if t is not None:
            batch.set_tuning(p, **{k: t.get(k, 0) for k in DEFAULT})
            n += 1
    return n
