"""Measuring autotuner for the sequential part of the path.

The forward and costate sweeps are a blocked two-level scan (block products
of length L, a sequential sweep over the N / L blocks, parallel passes
inside the blocks).  Their cost depends on L, on the padded dimension and
on the number of columns in ways that launch overheads, occupancy and
cache reuse decide, so the interval and the kernel variant of each sweep
are chosen by timing them on the problem itself: for every candidate L a
handle is built, each sweep is timed in the applicable variants (padded
d >= 80: per-block workgroups or per-step launches; smaller d: one
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

from .qoc import Problem

SWEEPS = ["fwd_blocks", "fwd_replay", "bwd_blocks", "bwd_pairs"]


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
        variants = (1, 2) if dp >= 80 else (1, 3)
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
            times[variant] = {ph: prof[ph][0] / reps for ph in SWEEPS + ["blockprod"]}
        h.close()
        choice = [min(variants, key=lambda v: times[v][ph]) for ph in SWEEPS]
        total = times[1]["blockprod"] + sum(times[v][ph] for v, ph in zip(choice, SWEEPS))
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
