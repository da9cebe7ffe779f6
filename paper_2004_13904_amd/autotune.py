"""Launch autotuner for the operator's column passes.

The only free launch parameters of a handle are the layer-group counts of the two column
passes (``ff_set_tuning``): more groups give more waves but more partial sums (G) or more
forward transforms (G^T).  ``autotune`` times every candidate on the caller's own vectors with
HIP events, keeps the fastest, and caches the choice in a JSON file keyed by the embedding,
layer count, survey size, dtype and batch width.
"""
from __future__ import annotations

import json
import os

import torch

CACHE = os.environ.get("FASTFOCUS_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "fastfocus_tune.json"))


def _key(op, k):
    s = op.survey
    return f"{op.nfft[0]}x{op.nfft[1]}:nz{op.nz}:s{s['sx']}x{s['sy']}:n{op.nx}x{op.ny}:{op.dtype}:k{k}"


def _candidates(nz):
    c = sorted({1, 2, 3, 4, 5, 8, 10, nz} & set(range(1, nz + 1)))
    return c


def _time(fn, reps=20):
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(op, x, d, cache=CACHE, use_cache=True):
    """Pick lg_G and lg_GT for op on vectors x (n values or k x n) and d (m values or k x m).
    Returns the chosen tuning dict (also applied to op)."""
    k = x.shape[0] if x.dim() == 2 else 1
    key = _key(op, k)
    table = {}
    if use_cache and cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if key in table:
        op.set_tuning(**table[key])
        return table[key]
    batched = x.dim() == 2
    G = (lambda: op.G_block(x)) if batched else (lambda: op.G(x))
    GT = (lambda: op.G_block(d, transpose=True)) if batched else (lambda: op.GT(d))
    cur = op.tuning
    best_g = min(_candidates(op.nz), key=lambda lg: (op.set_tuning(lg_G=lg, lg_GT=cur["lg_GT"]), _time(G))[1])
    best_t = min(_candidates(op.nz), key=lambda lg: (op.set_tuning(lg_G=best_g, lg_GT=lg), _time(GT))[1])
    choice = {"lg_G": int(best_g), "lg_GT": int(best_t)}
    op.set_tuning(**choice)
    if cache:
        table[key] = choice
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return choice
