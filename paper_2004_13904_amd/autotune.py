"""Launch autotuner of a handle: FFT stage plans, tile shapes and batch schedule.

The free launch parameters of a handle (``ff_set_tuning``) are:

* ``fft_plan_x``, ``fft_plan_y``: stage plans of the row (NX-point) and column (NY-point)
  transforms of the 2-D DFT taken as 1-D transforms (Appendix A of the paper): radix-8 stages with
  the radix-4 or radix-2 stage last (0) or first (1), or radix-4 stages (2); only the plans that
  differ for the size are tried;
* ``lg_G``, ``lg_GT``: layer groups of the two column passes (more groups give more waves but more
  partial sums for G, more forward transforms for G^T);
* ``row_tile``: transforms per row-pass block (automatic, one, two, four, or the largest that fits LDS);
* ``batch`` and ``col_batched`` (block applies only): vectors per launch, and the column-pass
  tile (G: 8 vectors per block with one whole vector per wave group, or 4 vectors per block with
  the layers split over its wave groups, or one vector per block).

``autotune`` times candidates on the caller's own vectors with HIP events (one G plus one G^T
per trial), by coordinate descent over the parameters in that order, keeps the fastest, and
caches the choice in a JSON file keyed by (NX, NY, nz, k, dtype).
"""
from __future__ import annotations

import json
import os

import torch

CACHE = os.environ.get("FASTFOCUS_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "fastfocus_tune.json"))


def _key(op, k):
    return f"NX{op.nfft[0]}:NY{op.nfft[1]}:nz{op.nz}:k{k}:{op.dtype}"


def fft_plans(n):
    """The stage plans that differ for an n-point transform: plan 1 is plan 0 when n is a power
    of 8 (no radix-4 or radix-2 stage to move)."""
    return [0, 2] if n.bit_length() % 3 == 1 else [0, 1, 2]


def _lg_candidates(nz):
    return sorted({1, 2, 3, 4, 5, 8, 10, nz} & set(range(1, nz + 1)))


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


def candidates(op, batched):
    """The values tried for each tuning key (dict key -> list), in search order."""
    c = {"fft_plan_x": fft_plans(op.nfft[0]), "fft_plan_y": fft_plans(op.nfft[1]),
         "lg_G": _lg_candidates(op.nz), "lg_GT": _lg_candidates(op.nz), "row_tile": [0, 1, 2, 3, 4]}
    if batched:
        bmax = op.batch_max
        c["batch"] = sorted({b for b in (4, 8, 16, 32, 64, bmax) if b <= bmax})
        c["col_batched"] = [2, 1, 0]
    return c


def autotune(op, x, d, cache=CACHE, use_cache=True, reps=20):
    """Pick the launch tuning of op for vectors x (n values or k x n) and d (m values or k x m).
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
        return op.tuning
    batched = x.dim() == 2
    if batched:
        def pair():
            op.G_block(x)
            op.G_block(d, transpose=True)
    else:
        def pair():
            op.G(x)
            op.GT(d)
    for name, values in candidates(op, batched).items():
        best, best_t = None, None
        for v in values:
            op.set_tuning(**{name: v})
            t = _time(pair, reps)
            if best_t is None or t < best_t:
                best, best_t = v, t
        op.set_tuning(**{name: best})
    choice = op.tuning
    if cache:
        table[key] = choice
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return choice
