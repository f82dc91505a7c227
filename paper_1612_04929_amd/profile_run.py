"""Run a few cost + gradient calls of a named synthetic workload, for a
profiler to attach to (rocprofv3 --kernel-trace --stats -- python3 -m
paper_1612_04929_amd.profile_run ...).  Device-resident inputs; prints the
per-call time of the timed calls and the handle's diagnostics.

  --config c2|c3|c4          the workload (workloads.make_config)
  --propagation matrix|action
  --precision fp32|fp64|bf16x3
  --segments S               memory-lean mode with S time segments
  --calls K --warmup W
"""
import argparse
import json
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c4")
    ap.add_argument("--propagation", default="matrix", choices=["matrix", "action"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--segments", type=int, default=1)
    ap.add_argument("--checkpoint-every", type=int, default=0)
    ap.add_argument("--calls", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import numpy as np
    import torch

    import workloads
    from paper_1612_04929_amd import qoc

    prob = workloads.make_config(args.config)
    seg = -(-prob.N // args.segments) if args.segments > 1 else 0
    h = qoc.Problem(prob, precision=args.precision, propagation=args.propagation,
                    checkpoint_every=args.checkpoint_every, segment_steps=seg)
    dev = torch.device("cuda:0")
    u = torch.from_numpy(np.ascontiguousarray(prob.u)).to(dev)
    out = torch.zeros(2 + prob.N, dtype=torch.float64, device=dev)
    grad = torch.zeros(max(1, prob.M * prob.N), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev).cuda_stream

    def call():
        h.cost_grad_device(u.data_ptr(), out.data_ptr(), grad.data_ptr(), st)

    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.calls):
        call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, args.calls)
    info = h.info()
    h.close()
    print(json.dumps(dict(workload=prob.name, propagation=args.propagation,
                          precision=args.precision, ms_per_call=ms, calls=args.calls,
                          p=info["p"], n=info["n"], segments=info["segments"],
                          device_bytes=info["device_bytes"], C_fid=float(out[1].item()))),
          flush=True)


if __name__ == "__main__":
    main()
