"""Stencil-only workload for hardware-counter runs.

    python paper_2609_37049_amd/profile_stencil.py [--dims 16x16x16x32] [--nrhs 32]
                                                   [--prec bf16|f32|f64] [--reps 10] [--solver-iters 20]
                                                   [--tile Y,T]

Launches the Wilson-clover stencil on native blocks of random spinors in the
launch configuration the solver uses (nrhs right-hand sides per launch, LDS
staging as the library chooses).  Then, with --solver-iters K > 0, runs K
inner iterations of the mixed-precision BiCGStab (reliable updates) on nrhs
random right-hand sides with HIP graphs off, so that every stencil launch the solver makes
(with its dot-product epilogues) is an ordinary dispatch a counter run can
see.  --tile sets the tile of the site order (y rows, timeslices; the
autotuner's choice in a benchmark run) instead of the default rule.  Last comes a plain 256 MiB device-to-device copy whose byte counts
calibrate the FETCH_SIZE / WRITE_SIZE counters.  Prints the algorithmic
bytes per stencil launch.
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
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--prec", default="bf16", choices=["bf16", "f32", "f64"])
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--solver-iters", type=int, default=20)
    ap.add_argument("--tile", default="")
    args = ap.parse_args()
    dims = tuple(int(v) for v in args.dims.split("x"))
    prec = {"f64": d.F64, "f32": d.F32, "bf16": d.BF16}[args.prec]
    n = args.nrhs
    U = synth.gauge_field(dims, 0.25, 2)
    ctx = d.Context(dims, (1, 1, 1, -1))
    ctx.gauge_set(U)
    ctx.clover_setup(0.125, 1.5)
    if args.tile:
        ty, tt = (int(v) for v in args.tile.split(","))
        ctx.set_option(d.OPT_TILE_Y, ty)
        ctx.set_option(d.OPT_TILE_T, tt)
    nb = ctx.native_bytes(prec, n)
    x = (torch.rand(nb // 4, device="cuda") - 0.5).view(torch.uint8)
    if prec == d.BF16:
        x = torch.randint(-2 ** 15, 2 ** 15, (nb // 2,), dtype=torch.int16, device="cuda").view(torch.uint8)
        # keep the bf16 payload finite: clear the exponent field's top bit of every half-word
        x.view(torch.int16).bitwise_and_(0x3fff)
    y = torch.empty_like(x)
    for _ in range(args.reps):
        ctx.dirac_apply_native(None, prec, x, y, n)
    torch.cuda.synchronize()
    if args.solver_iters > 0 and prec != d.F64:
        ctx.set_option(d.OPT_GRAPHS, 0)
        g = torch.Generator(device="cuda").manual_seed(5)
        b = torch.complex(torch.randn((n, ctx.V, 4, 3), generator=g, dtype=torch.float64, device="cuda"),
                          torch.randn((n, ctx.V, 4, 3), generator=g, dtype=torch.float64, device="cuda"))
        P = ctx.params(method=d.BICGSTAB_RU, tol=1e-10, max_iter=args.solver_iters, inner_prec=prec,
                       rhs_block=n, fallback=0, check_every=args.solver_iters)
        ctx.solve_multi_rhs(b, P, allow_noconv=True)
        torch.cuda.synchronize()
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    sp = {d.F64: 8, d.F32: 4, d.BF16: 2}[prec]
    sg = 8 if prec == d.F64 else 4
    V = ctx.V
    alg_read = V * (n * 24 * sp + 144 * sg)
    alg_write = V * n * 24 * sp
    print("stencil %s %s nrhs %d tile %d,%d: algorithmic read %d B, write %d B per launch; copy %d B read + %d B write"
          % (args.dims, args.prec, n, ctx.get_option(d.OPT_TILE_Y), ctx.get_option(d.OPT_TILE_T), alg_read, alg_write,
             src.numel() * 4, src.numel() * 4), flush=True)


if __name__ == "__main__":
    main()
