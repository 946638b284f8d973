"""Scatter autotuner.

The scatter's tiles (in-plane nonzeros per block), set slots per chunk and the
number of blocks the thickness chunking aims at change its speed, not its
values.  `tune` times the scatter of lam_assemble (HIP events around the
kernel) for a short list of tunings on one laminate and returns the fastest;
tunings are cached per laminate class (in-plane degrees, thickness degree, set
mode) in a JSON file, which `lookup` reads.  Running this module on a GPU
tunes the plates of the benchmark and the classes of the uneven batch:

    python -m paper_1905_05417_amd.autotune OUT.json
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import torch

from . import lamasm as L

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.json")

CANDIDATES = ([{}] + [{"tile_k": tk} for tk in (32, 48, 64)]
              + [{"target_blocks": b} for b in (1536, 3072, 12288, 24576)]
              + [{"tile_k": 48, "target_blocks": 12288}, {"tile_k": 64, "target_blocks": 12288}])


def class_key(lam, set_mode: str) -> str:
    """In-plane degrees, thickness degree, set mode and log2 of the row count."""
    return "p%dx%d_q%d_%s_r%d" % (int(lam.p1), int(lam.p2), int(lam.q), set_mode,
                                  int(round(np.log2(max(lam.n_rows, 1)))))


def time_scatter(lam, set_mode: str, tuning: dict, reps: int = 5, vals=None) -> float:
    """Mean scatter milliseconds of lam_assemble with this tuning (into `vals` if given)."""
    plan = L.Plan(lam, set_mode=set_mode, tuning=tuning)
    C = torch.tensor(np.asarray(lam.C), device="cuda")
    th = torch.tensor(np.asarray(lam.theta), device="cuda")
    own = vals is None
    if own:
        vals = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    plan.assemble(C, th, out=vals)
    torch.cuda.synchronize()
    L.profile_enable(True)
    L.profile_read()
    for _ in range(reps):
        plan.assemble(C, th, out=vals)
    ms, n = L.profile_read()["assemble"]
    L.profile_enable(False)
    del plan
    if own:
        del vals
        torch.cuda.empty_cache()
    return ms / max(n, 1)


def tune(lam, set_mode: str = "bucket", candidates=None, reps: int = 5, rounds: int = 2):
    """(best tuning, [(tuning, ms), ...]) over the candidates; infeasible ones are skipped.

    The scatter's speed also depends on where its output lands in device
    memory, so every candidate writes into the same buffer, and the candidates
    are timed in `rounds` interleaved rounds (the minimum counts)."""
    cands = list(candidates or CANDIDATES)
    nnz = L.Plan(lam, set_mode=set_mode).nnz
    vals = torch.empty(nnz, dtype=torch.float64, device="cuda")
    best_ms = {}
    for _ in range(rounds):
        for i, cand in enumerate(cands):
            try:
                ms = time_scatter(lam, set_mode, cand, reps, vals=vals)
            except L.LamError:
                continue
            best_ms[i] = min(best_ms.get(i, ms), ms)
    del vals
    torch.cuda.empty_cache()
    results = [(cands[i], best_ms[i]) for i in sorted(best_ms)]
    best = min(results, key=lambda r: r[1])[0]
    return best, results


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def lookup(lam, set_mode: str, cache: dict | None = None):
    """Cached tuning of the laminate's class, or None (automatic)."""
    cache = load_cache() if cache is None else cache
    key = class_key(lam, set_mode)
    rec = cache.get(key)
    if rec is None:  # nearest size of the same degrees and set mode
        stem, size = key.rsplit("_r", 1)
        near = [(abs(int(k.rsplit("_r", 1)[1]) - int(size)), k) for k in cache if k.rsplit("_r", 1)[0] == stem]
        if near:
            rec = cache[min(near)[1]]
    return None if rec is None else rec["tuning"]


def _main(out_path: str):
    from . import workloads as W
    torch.cuda.init()
    L.lib()
    jobs = [(W.config_p2_64x64_32ply(), "bucket"), (W.config_p3_128x128_128ply(), "bucket"),
            (W.config_adjoint_p2_96x96_64ply(), "bucket")]
    # uneven batch: one mid-size member per class
    by_class = {}
    for lam in W.batch_laminates():
        by_class.setdefault(class_key(lam, "bucket"), []).append(lam)
    for key, lams in sorted(by_class.items()):
        if len(lams) >= 8:  # the well-populated size classes
            jobs.append((lams[len(lams) // 2], "bucket"))
    cache = load_cache(out_path)
    for lam, mode in jobs:
        key = class_key(lam, mode)
        if key in cache:
            continue
        best, results = tune(lam, mode)
        cache[key] = {"tuning": best, "tuned_on": lam.name,
                      "ms": {json.dumps(t, sort_keys=True): round(ms, 5) for t, ms in results}}
        print(key, lam.name, "best", best, "%.4f ms" % min(ms for _, ms in results),
              "auto %.4f ms" % results[0][1], flush=True)
        with open(out_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    _main(sys.argv[1] if len(sys.argv) > 1 else DEFAULT_CACHE)
