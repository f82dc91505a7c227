"""Measuring autotuners: the product tile shape (the padding multiple of d)
and the sequential part of the path.

Tile shape: padding d to a multiple of 64 runs every product on 64 x 64
MFMA tiles at the price of more zero padding; a multiple of 16 keeps the
16- / 32-wide tiles (and the LDS chains for d <= 48).  Which wins depends
on d (the padding factor (d64 / d16)^3 against the tile efficiency), so
:func:`tune_tiles` times both on the problem and caches the choice by
(architecture, d, S, M, precision).

Sequential part:

The forward and costate sweeps are a blocked two-level scan (block products
of length L, a sequential sweep over the N / L blocks, parallel passes
inside the blocks).  Their cost depends on L, on the padded dimension and
on the number of columns in ways that launch overheads, occupancy and
cache reuse decide, so the interval and the kernel variant of each sweep
are chosen by timing them on the problem itself: for every candidate L a
handle is built, each sweep is timed in the applicable variants (padded
d >= 80: per-block workgroups or per-step launches with the products on
the VALU or on the MFMA; smaller d: one
wavefront or a four-wavefront LDS-staged workgroup; FP32 padded d 64 ..
128 also one 8 d_pad-thread chain workgroup per block; padded d 16 also
longer blocks, whose in-block passes run over sub-blocks) with the library's
per-phase HIP events, and the L that minimises block products plus the
best variant of each sweep wins.  Other phases do not depend on these
choices.
"""
from __future__ import annotations

import math
import time

import json
import os

from .qoc import Problem

SWEEPS = ["fwd_blocks", "fwd_replay", "bwd_blocks", "bwd_pairs"]

# Tile-shape choices measured so far, keyed by (architecture, d, S, M,
# precision); persisted as JSON so that later processes reuse them.
_TILE_CACHE = None


def _cache_path():
    return os.environ.get("QOC_TUNE_CACHE", os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1612_04929_amd", "tiles.json"))


def _tile_cache():
    global _TILE_CACHE
    if _TILE_CACHE is None:
        try:
            with open(_cache_path()) as f:
                _TILE_CACHE = json.load(f)
        except (OSError, ValueError):
            _TILE_CACHE = {}
    return _TILE_CACHE


def tile_key(prob, precision, device=0):
    import torch
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    return f"{arch}|d={prob.d}|S={prob.S}|M={prob.M}|{precision}"


def pad_candidates(d):
    """Padding multiples that change the tiles: 16 (16 / 32-wide tiles, the
    LDS chains up to 48) and 64 (64 x 64 MFMA tiles) when they differ."""
    r16, r64 = (d + 15) // 16 * 16, (d + 63) // 64 * 64
    return [16, 64] if d > 32 and r64 != r16 else [16]


def tune_tiles(prob, precision="fp32", steps=256, reps=3, device=0):
    """Padding multiple (the product tile shape) for a problem: every
    candidate of pad_candidates is timed on the first `steps` steps (a whole
    cost + gradient call, tiles, sweeps and derivative included), the
    fastest kept, and the choice cached by (architecture, d, S, M,
    precision).  Returns dict(pad_multiple, ms per candidate, cached)."""
    import numpy as np
    import torch
    cands = pad_candidates(prob.d)
    key = tile_key(prob, precision, device)
    cache = _tile_cache()
    if len(cands) == 1:
        return dict(pad_multiple=cands[0], ms={}, cached=False)
    if key in cache:
        return dict(pad_multiple=cache[key]["pad_multiple"], ms=cache[key]["ms"], cached=True)
    q = prob.with_steps(min(prob.N, steps))
    dev = torch.device(f"cuda:{device}")
    u = torch.from_numpy(np.ascontiguousarray(q.u, dtype=np.float64)).to(dev)
    out = torch.zeros(2 + q.N, dtype=torch.float64, device=dev)
    grad = torch.zeros(max(1, q.M * q.N), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    ms = {}
    for pm in cands:
        h = Problem(q, precision=precision, device=device, pad_multiple=pm)
        h.cost_grad_device(u.data_ptr(), out.data_ptr(), grad.data_ptr(), st)
        torch.cuda.synchronize(dev)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            h.cost_grad_device(u.data_ptr(), out.data_ptr(), grad.data_ptr(), st)
            torch.cuda.synchronize(dev)
            best = min(best, time.perf_counter() - t0)
        h.close()
        ms[str(pm)] = best * 1e3
    choice = int(min(ms, key=ms.get))
    cache[key] = dict(pad_multiple=choice, ms=ms)
    try:
        os.makedirs(os.path.dirname(_cache_path()), exist_ok=True)
        with open(_cache_path(), "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return dict(pad_multiple=choice, ms=ms, cached=False)


def candidate_intervals(N: int, d: int | None = None):
    base = 1 << max(0, round(math.log2(max(1.0, math.sqrt(N)))))
    cands = {max(1, base // 4), max(1, base // 2), base, base * 2}
    if d is not None and d <= 16:
        # padded d 16: the in-block passes run over sub-blocks of 8 steps in
        # parallel, which makes longer blocks worth timing
        cands.add(min(base * 4, 64))
    return sorted(c for c in cands if c <= max(1, N))


def tune(prob, precision="fp32", intervals=None, reps=3, device=0, **kw):
    """Returns dict(checkpoint_every=L, sweep=[v0, v1, v2, v3], table=[...],
    seconds=tuning time).  `prob` as for :class:`Problem`."""
    import numpy as np
    import torch

    t0 = time.perf_counter()
    dev = torch.device(f"cuda:{device}")
    u = torch.from_numpy(np.ascontiguousarray(prob.u, dtype=np.float64)).to(dev)
    out = torch.zeros(2 + prob.N, dtype=torch.float64, device=dev)
    grad = torch.zeros(max(1, prob.M * prob.N), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    table = []
    for L in intervals or candidate_intervals(prob.N, getattr(prob, "d", None)):
        h = Problem(prob, precision=precision, checkpoint_every=L, device=device, **kw)
        times = {}
        dp = h.info()["d_pad"]
        variants = (1, 2, 5) if dp >= 80 else (1, 3)
        if precision != "fp64" and 64 <= dp <= 128:
            variants += (4,)  # chain workgroups (FP32 chains)
        for variant in variants:
            h.set_sweep(-1, variant)
            h.cost_grad_device(u.data_ptr(), out.data_ptr(), grad.data_ptr(), st)
            torch.cuda.synchronize(dev)
            h.profile_enable(True)
            h.profile_read(reset=True)
            for _ in range(reps):
                h.cost_grad_device(u.data_ptr(), out.data_ptr(), grad.data_ptr(), st)
            prof = h.profile_read(reset=True)
            h.profile_enable(False)
            times[variant] = {ph: prof[ph][0] / reps for ph in SWEEPS + ["blockprod", "cost"]}
        h.close()

        def score(v, ph):
            # the single-wavefront backward block sweep (padded d 16) runs
            # lambda_N, the fidelity and the penalties inside its own launch
            # instead of the cost launch: that launch counts with it
            return times[v][ph] + (times[v]["cost"] if ph == "bwd_blocks" else 0.0)

        choice = [min(variants, key=lambda v: score(v, ph)) for ph in SWEEPS]
        total = times[1]["blockprod"] + sum(score(v, ph) for v, ph in zip(choice, SWEEPS))
        table.append(dict(L=L, sweep=choice, ms=total,
                          phases={ph: {v: times[v][ph] for v in variants} for ph in SWEEPS}))
    best = min(table, key=lambda r: r["ms"])
    return dict(checkpoint_every=best["L"], sweep=best["sweep"], table=table,
                seconds=time.perf_counter() - t0)


def apply(handle: Problem, cfg) -> None:
    """Set the tuned sweep variants on a handle built with
    checkpoint_every=cfg['checkpoint_every']."""
    for which, variant in enumerate(cfg["sweep"]):
        handle.set_sweep(which, variant)
