"""Many independent control problems per optimizer iteration.

A :class:`Batch` holds one libqoc handle per instance (uneven d, N, M), the
instances' amplitudes and gradients packed back to back in flat device
buffers (each instance's M x N block a contiguous slice), the Adam moments
and step count beside them, and the outputs.  One iteration enqueues
``qoc_cost_grad_batched`` for every instance, split over a few streams
(default priority) forked from and joined back into the current stream,
then one ``qoc_adam_step`` over all amplitudes (the library's Adam kernel;
torch only allocates the buffers).  Handles whose padded d is 32 or more get a fixed
(p, n) chosen from their initial theta_max times a margin: from 64 on no
call then needs a host round trip, and from 32 on the per-step derivative
runs as batched tile products (padded d 16 choose (p, n) on the device);
the device checks a fixed pair against the tolerance on every call
(QOC_WARN_TAYLOR, see :meth:`taylor_warnings`), and :meth:`refresh`
re-chooses pairs that no longer hold.  The whole iteration can then be
captured in one HIP graph and replayed.
"""
from __future__ import annotations

import ctypes as C
import heapq
import math

import numpy as np
import torch

from . import qoc


def taylor_ok(p, n, theta, tol):
    """The truncation bound of the (p, n) rule, 2^n x^(p+1)/(p+1)! e^x <= tol
    with x = theta / 2^n (Sec. III), for a given pair."""
    x = math.ldexp(theta, -n)
    return math.ldexp(1.0, n) * x ** (p + 1) / math.factorial(p + 1) * math.exp(x) <= tol


class Batch:
    def __init__(self, problems, precision="fp32", streams=4, device=0, margin=1.1,
                 lr=1e-2, betas=(0.9, 0.999), eps=1e-8, tune_tiles=False):
        self.dev = torch.device(f"cuda:{device}")
        self.problems = list(problems)
        # tile shape per instance (padding multiple of d), measured and cached
        # by (architecture, d, S, M, precision) when tune_tiles is set
        self.pads = [16] * len(self.problems)
        self.tile_tuning = {}
        if tune_tiles:
            from . import tune
            for i, p in enumerate(self.problems):
                r = tune.tune_tiles(p, precision=precision, device=device)
                self.pads[i] = r["pad_multiple"]
                self.tile_tuning[tune.tile_key(p, precision, device)] = r
        self.handles = [qoc.Problem(p, precision=precision, device=device, pad_multiple=pm)
                        for p, pm in zip(self.problems, self.pads)]
        f64 = torch.float64
        sizes = [max(1, p.M * p.N) for p in self.problems]
        offs = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
        self.n_amp = int(offs[-1])
        u0 = np.zeros(self.n_amp)
        for p, o in zip(self.problems, offs):
            u0[o: o + p.M * p.N] = np.asarray(p.u, dtype=np.float64).ravel()
        self.u_flat = torch.tensor(u0, dtype=f64, device=self.dev)
        self.g_flat = torch.zeros(self.n_amp, dtype=f64, device=self.dev)
        self.m_flat = torch.zeros(self.n_amp, dtype=f64, device=self.dev)
        self.v_flat = torch.zeros(self.n_amp, dtype=f64, device=self.dev)
        self.t_step = torch.zeros(1, dtype=f64, device=self.dev)
        self.lr, self.betas, self.eps = float(lr), (float(betas[0]), float(betas[1])), float(eps)
        self.u = [self.u_flat[o: o + p.M * p.N].view(p.M, p.N)
                  for p, o in zip(self.problems, offs)]
        self.grad = [self.g_flat[o: o + s] for o, s in zip(offs, sizes)]
        self.out = [torch.zeros(2 + p.N, dtype=f64, device=self.dev) for p in self.problems]
        self.total_steps = int(sum(p.N for p in self.problems))
        # initial (p, n): one call per instance, then fix the pair of the
        # instances that would otherwise read theta_max back on the host
        st = torch.cuda.current_stream(self.dev).cuda_stream
        for h, u, o, g in zip(self.handles, self.u, self.out, self.grad):
            h.cost_grad_device(u.data_ptr(), o.data_ptr(), g.data_ptr(), st)
        torch.cuda.synchronize(self.dev)
        self.pn = []
        self.tol = 1e-15 if precision == "fp64" else 1e-10
        for h in self.handles:
            inf = h.info()
            if inf["d_pad"] >= 32:
                p, n = h.pair_for(inf["theta_max"] * margin)
                h.set_taylor(p, n)
                self.pn.append((p, n))
            else:
                self.pn.append(None)
        # longest-processing-time assignment of instances to streams
        cost = [p.N * (max(16, (p.d + 15) // 16 * 16) ** 3 + 16 ** 3 * 8) for p in self.problems]
        nstr = max(1, int(streams))
        heap = [(0.0, k) for k in range(nstr)]
        self.groups = [[] for _ in range(nstr)]
        for i in sorted(range(len(cost)), key=lambda i: -cost[i]):
            load, k = heapq.heappop(heap)
            self.groups[k].append(i)
            heapq.heappush(heap, (load + cost[i], k))
        self.groups = [g for g in self.groups if g]
        self.streams = [torch.cuda.Stream(self.dev) for _ in self.groups]
        self._fork = torch.cuda.Event()
        self._join = [torch.cuda.Event() for _ in self.groups]
        self._arrays = []
        for g in self.groups:
            B = len(g)
            arr = lambda xs: (C.c_void_p * B)(*[C.c_void_p(int(x)) for x in xs])
            self._arrays.append((B, (C.c_void_p * B)(*[self.handles[i]._h for i in g]),
                                 arr([self.u[i].data_ptr() for i in g]),
                                 arr([self.out[i].data_ptr() for i in g]),
                                 arr([self.grad[i].data_ptr() for i in g])))
        self.graph = None

    # ------------------------------------------------------------------
    def cost_grad(self):
        """Enqueue cost + gradient of every instance (multi-stream fork/join)."""
        lib = qoc.load()
        main = torch.cuda.current_stream(self.dev)
        self._fork.record(main)
        for s, ev, (B, hs, us, outs, grads) in zip(self.streams, self._join, self._arrays):
            s.wait_event(self._fork)
            qoc._check(lib.qoc_cost_grad_batched(B, hs, us, outs, grads,
                                                 C.c_void_p(s.cuda_stream)))
            ev.record(s)
        for ev in self._join:
            main.wait_event(ev)

    def cost_grad_serial(self):
        """Per-instance calls on the current stream (the unbatched baseline)."""
        st = torch.cuda.current_stream(self.dev).cuda_stream
        for h, u, o, g in zip(self.handles, self.u, self.out, self.grad):
            h.cost_grad_device(u.data_ptr(), o.data_ptr(), g.data_ptr(), st)

    def adam(self):
        """One Adam step over every instance's amplitudes (qoc_adam_step)."""
        qoc.adam_step(self.n_amp, self.u_flat.data_ptr(), self.g_flat.data_ptr(),
                      self.m_flat.data_ptr(), self.v_flat.data_ptr(), self.t_step.data_ptr(),
                      self.lr, self.betas, self.eps,
                      torch.cuda.current_stream(self.dev).cuda_stream)

    def iteration(self, serial=False):
        (self.cost_grad_serial if serial else self.cost_grad)()
        self.adam()

    def capture(self, warmup=3):
        """Capture one iteration (all cost + gradient calls and the Adam
        update) in a HIP graph; warm-up iterations run first on a side
        stream."""
        side = torch.cuda.Stream(self.dev)
        side.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.iteration()
        torch.cuda.current_stream(self.dev).wait_stream(side)
        torch.cuda.synchronize(self.dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.iteration()
        torch.cuda.synchronize(self.dev)

    def replay(self):
        self.graph.replay()

    # ------------------------------------------------------------------
    def costs(self):
        return np.array([float(o[0]) for o in self.out])

    def refresh(self, margin=1.25, ahead=1.1):
        """Re-choose the fixed (p, n) of every instance whose pair missed the
        tolerance on its last call or would miss it at `ahead` times its
        current theta_max (from `margin` times theta_max), then re-capture
        the graph if any pair changed.  Synchronises; run it between timed
        replays.  Returns the number of instances changed."""
        torch.cuda.synchronize(self.dev)
        changed = 0
        for i, h in enumerate(self.handles):
            inf = h.check_last()  # raises on a clamped pair (QOC_WARN_NO_PAIR)
            if self.pn[i] is None:
                continue
            tol = self.tol
            p, n = self.pn[i]
            if (inf["flags"] & qoc.QOC_WARN_TAYLOR) or not taylor_ok(p, n, inf["theta_max"] * ahead,
                                                                    tol):
                pn = h.pair_for(inf["theta_max"] * margin)
                if pn != (p, n):
                    h.set_taylor(*pn)
                    self.pn[i] = pn
                    changed += 1
        if changed and self.graph is not None:
            self.graph = None
            self.capture(warmup=1)
        return changed

    def taylor_warnings(self):
        """Indices of instances whose fixed (p, n) missed the tolerance on
        their last call."""
        return [i for i, h in enumerate(self.handles) if h.info()["flags"] & qoc.QOC_WARN_TAYLOR]

    def close(self):
        for h in self.handles:
            h.close()
        self.handles = []
