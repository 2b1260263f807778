"""Network-only workload for kernel traces and hardware-counter runs.

    python paper_2609_37049_amd/profile_nn.py [--dims 16x16x16x32] [--nrhs 8] [--reps 5] [--backward]

Creates the gauge-covariant network on a synthetic gauge field (links
exp(i 0.25 sum r_a T_a), seed 2), applies it to nrhs Gaussian fields `reps`
times (three layer launches each) and, with --backward, runs one backward pass
(three weight-gradient contractions and two adjoint layers).  Prints the
matrix-core work of the forward pass and the time per application measured
with HIP events.
"""
import argparse
import os
import sys

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
import paper_2609_37049_amd as d  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="16x16x16x32")
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--backward", action="store_true")
    args = ap.parse_args()
    dims = tuple(int(v) for v in args.dims.split("x"))
    n = args.nrhs
    U = synth.gauge_field(dims, 0.25, 2)
    ctx = d.Context(dims, (1, 1, 1, -1))
    ctx.gauge_set(U)
    net = d.Net(ctx, 16, 7)
    g = torch.Generator().manual_seed(3)
    x = torch.complex(torch.randn((n, ctx.V, 4, 3), generator=g, dtype=torch.float64),
                      torch.randn((n, ctx.V, 4, 3), generator=g, dtype=torch.float64)).cuda()
    net.apply(x)
    torch.cuda.synchronize()
    ctx.profile_reset()
    ctx.profile_enable(True)
    for _ in range(args.reps):
        net.apply(x)
    ctx.profile_enable(False)
    nl, ms, fl = ctx.profile_get(d.K_NN)
    per = ms / args.reps
    print("network %s, %d RHS: %d layer launches, %.3f ms per application (%.3f ms per RHS), "
          "%.1f TFLOP/s of matrix-core work (%.1f%% of 2.5 PFLOP/s dense BF16)"
          % (args.dims, n, nl, per, per / n, fl / (ms / 1e3) / 1e12, 100 * fl / (ms / 1e3) / 2.5e15), flush=True)
    if args.backward:
        gw, gi = net.backward(x, x)
        torch.cuda.synchronize()
        print("backward done", flush=True)


if __name__ == "__main__":
    main()
