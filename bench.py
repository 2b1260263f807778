"""Benchmark of the hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--inner bf16|f32] [--method ru|dc] [--inner-tol D]
                    [--workload batch_24x24x24x48|prec_16x16x16x32|prod_32x32x32x64|learned_24x24x24x48]
                    [--nv-per-step N] [--nn-pairs P] [--nn-steps S]
                    [--no-cpu-baseline] [--no-legs]

Workload (default): the batching configuration, a 24^3 x 48 lattice
(synthetic links exp(i 0.25 sum r_a T_a), 5 APE steps alpha = 0.5 for the
Laplacian, Wilson-clover kappa = 0.126, csw = 1.6, antiperiodic time, Nv = 64
eigenvectors per timeslice, domains 6 x 6 x 8 x 12), solved to true relative
residual 1e-10 by BiCGStab with BF16-stored, FP32-arithmetic inner solves on
the even-odd Schur complement and FP64 reliable updates (--method dc: inside
FP64 defect correction), 64 right-hand sides per launch fed from one queue.
--workload prec_16x16x16x32 runs the same step on the 16^3 x 32 precision
shape (kappa = 0.125, csw = 1.5, Nv = 32, domains 4^3 x 8).
--workload prod_32x32x32x64 times a stated subset of the production shape
(32^3 x 64, four ensembles; see production_subset), and --workload
learned_24x24x24x48 the learned preconditioner's configuration (see
learned_form).

One step is one batch of the whole hot path: the four timeslices of one
multi-site packing set (one timeslice per temporal layer of the partition)
for one group of eigenvectors (16 of the 64 at 24^3 x 48, all 32 at
16^3 x 32) -- sources, full-operator solves (4 x 4 x group RHS), packed
domain-restricted solves (4 x group solves carrying 4 x 4 x group logical
RHS), perambulator projection, loops for five Gamma channels and their
Gamma-tilde (formed by the library), and the full / factorised / subtracted
correlators.  Steps cycle through the packing sets and eigenvector groups.
The value is logical RHS (full + restricted) per second over the timed steps,
with the full-operator and D_Lambda rates beside it; set-up (clover term,
APE, eigenvectors, autotuning) is timed once before and reported beside it.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "distillation RHS solved/s at rel. residual 1e-10; Dirac stencil HBM GB/s"
HBM_PEAK_GBPS = 8000.0
# FP32 vector peak: 256 CUs x 4 SIMDs x 32 lanes per cycle x 2 flop (FMA) x 2.4 GHz
# = 157.3 TFLOP/s.  A plain (non-packed) v_fmac_f32 issue-rate probe on the chip
# sustains about 96 TFLOP/s, which the bench reports beside it.
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12
VALU_FP32_FMAC_PROBE_TFLOPS = 96.0
# conventional Wilson-clover flop count per site and right-hand side: hopping 1320,
# clover 504, combination 48
FLOP_PER_SITE_RHS = 1872
STENCIL_SOURCES = ["paper_2609_37049_amd/csrc/stencil.hip", "paper_2609_37049_amd/csrc/spinor_io.h"]


def stencil_hash():
    h = hashlib.sha256()
    for p in STENCIL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel_tag):
    """HBM bytes per launch of the timed stencil, from committed rocprofv3 counter
    runs (FETCH_SIZE, WRITE_SIZE scaled by a plain-copy calibration); null when
    the kernel sources changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "stencil_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    ent = d.get(kernel_tag)
    if not ent or ent.get("source_hash") != stencil_hash():
        return None
    return ent.get("bytes_per_launch")


def traffic_key(kernel_tag, blk, lat, tile):
    """Key of the committed counter entry for a stencil family, block width,
    lattice and site-order tile (the counters depend on all four)."""
    return "%s/n%d/%s/tile%dx%d" % (kernel_tag, blk, lat, tile[0], tile[1])


MFMA_BF16_PEAK_TFLOPS = 2500.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def stencil_roofline(kernel_tag, nl, ms, by, sites, blk, traffic_key):
    """HBM roofline of a stencil family from event-timed launches: algorithmic
    bytes over time against the HBM peak, with the calibrated counter traffic
    (when the committed entry matches the sources) and the vector-ALU rate
    beside it.  The launches are bound on the memory side (L1 misses, each
    paying the L2 round trip); neither the ALUs nor HBM saturate."""
    avg_ms = ms / max(nl, 1)
    gbps = by / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    tflops = FLOP_PER_SITE_RHS * sites * blk / (avg_ms / 1e3) / 1e12 if avg_ms > 0 else 0.0
    traffic = load_traffic(traffic_key)
    return {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "traffic_gbps": round(traffic / (avg_ms / 1e3) / 1e9, 1) if traffic else None,
            "alu_tflops": round(tflops, 2), "alu_peak_tflops": round(VALU_FP32_PEAK_TFLOPS, 1),
            "alu_frac": round(tflops / VALU_FP32_PEAK_TFLOPS, 4),
            "alu_frac_of_fmac_probe": round(tflops / VALU_FP32_FMAC_PROBE_TFLOPS, 4),
            "kernel": kernel_tag + " (inner-precision Wilson-clover stencil, full operator, %d RHS per launch, %d sites)"
            % (blk, sites),
            "avg_launch_ms": round(avg_ms, 5), "launches_timed": nl,
            "alg_bytes_per_launch": round(by / max(nl, 1)),
            "flop_per_launch": FLOP_PER_SITE_RHS * sites * blk}


def stencil_at_batch_shape(d, inner, blk, iters=20):
    """The dominant stencil at the 24^3x48 batching shape, whose working set
    (over 1 GB per half-lattice vector at 64 right-hand sides) is far beyond the
    256 MB Infinity Cache: a short solve with reliable updates on blk random
    right-hand sides, every stencil launch event-timed.  Not part of value."""
    import torch
    import synth
    pre = synth.PRESETS["batch_24x24x24x48"]
    U = synth.gauge_field(pre.dims, pre.eps, pre.seed)
    ctx = d.Context(pre.dims, pre.bc, 0)
    ctx.gauge_set(U)
    ctx.clover_setup(pre.kappa, pre.csw)
    del U
    g = torch.Generator(device="cuda:0").manual_seed(31)
    b = torch.complex(torch.randn((blk, ctx.V, 4, 3), generator=g, device="cuda:0", dtype=torch.float64),
                      torch.randn((blk, ctx.V, 4, 3), generator=g, device="cuda:0", dtype=torch.float64))
    P = ctx.params(method=d.BICGSTAB_RU, tol=1e-10, max_iter=iters, inner_prec=inner, rhs_block=blk, fallback=0)
    ctx.solve_multi_rhs(b, P, allow_noconv=True)
    ctx.profile_reset()
    ctx.profile_stride(1)
    ctx.set_option(d.OPT_NARROW, 0)  # every timed launch at the block width
    ctx.profile_enable(True)
    ctx.solve_multi_rhs(b, P, allow_noconv=True)
    ctx.profile_enable(False)
    ctx.set_option(d.OPT_NARROW, 1)
    fam = d.K_STENCIL_EO_BF16 if inner == d.BF16 else d.K_STENCIL_EO_F32
    tag = "k_dslash_eo<%s>" % ("IOBF" if inner == d.BF16 else "IO32")
    nl, ms, by = ctx.profile_get(fam)
    tile = (ctx.get_option(d.OPT_TILE_Y), ctx.get_option(d.OPT_TILE_T))
    roof = stencil_roofline(tag, nl, ms, by, ctx.V // 2, blk, traffic_key(tag, blk, "24x24x24x48", tile))
    roof["lattice"] = "24x24x24x48"
    del b, ctx
    torch.cuda.empty_cache()
    return roof


def solver_comparison(ctx, d, Vev, inner, tuned, T, inner_tol=0.0):
    """The plain FP64 GPU solvers, the production mixed-precision batched
    solver and the learned-preconditioner solver on the same 16 distillation
    sources (timeslice 0, eigenvectors 0..3 x 4 spins) to true relative
    residual 1e-10.  Not part of the timed steps."""
    import torch
    V, Vs = ctx.V, ctx.Vs
    b = torch.zeros((16, V, 4, 3), dtype=torch.complex128, device="cuda:0")
    for i in range(4):
        for a in range(4):
            b[4 * i + a, :Vs, a, :] = Vev[0, i]
    out = {}

    def run(name, P, nb):
        bb = b[:nb].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = ctx.solve_multi_rhs(bb, P)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"rhs_per_s": round(nb / dt, 3), "rhs": nb, "iters": st[0].iters,
                     "fallback_used": max(s.fallback_used for s in st),
                     "worst_true_rel_residual": max(s.true_rel_residual for s in st)}
        print("comparison %s: %.2f RHS/s" % (name, nb / dt), file=sys.stderr, flush=True)

    run("cgnr_f64_1rhs_plain", ctx.params(method=d.CGNR_F64, tol=1e-10, rhs_block=1), 2)
    ctx.set_option(d.OPT_EO, 0)
    run("bicgstab_f64_1rhs_unpreconditioned", ctx.params(method=d.BICGSTAB_DC, tol=1e-10, inner_prec=d.F64,
                                                          rhs_block=1), 2)
    ctx.set_option(d.OPT_EO, 1)
    run("bicgstab_f64_1rhs_even_odd", ctx.params(method=d.BICGSTAB_DC, tol=1e-10, inner_prec=d.F64, rhs_block=1), 2)
    run("mixed_batched_bicgstab_defect_correction", ctx.params(method=d.BICGSTAB_DC, tol=1e-10, inner_prec=inner,
                                                               rhs_block=tuned), 16)
    run("mixed_batched_bicgstab_reliable_updates", ctx.params(method=d.BICGSTAB_RU, tol=1e-10, inner_prec=inner,
                                                               rhs_block=tuned, inner_tol=inner_tol), 16)
    net = d.Net(ctx, 16, 7)
    t0 = time.perf_counter()
    ts = net.train(64, snap_iters=(0, 16, 64, 192), batch=4, steps=100, lr=2e-3, seed=5)
    train_s = time.perf_counter() - t0
    ctx.profile_reset()
    ctx.profile_stride(1)
    ctx.profile_enable(True)
    run("mixed_batched_learned_fgmres16", ctx.params(method=d.FGMRES_NN, tol=1e-10, net=net, restart=16,
                                                     rhs_block=8), 8)
    ctx.profile_enable(False)
    nl, ms, fl = ctx.profile_get(d.K_NN)
    tf = fl / (ms / 1e3) / 1e12 if ms > 0 else 0.0
    out["mixed_batched_learned_fgmres16"].update({
        "train_pairs": ts.pairs, "train_steps": ts.steps, "train_loss_first": round(ts.first_loss, 4),
        "train_loss_final": round(ts.final_loss, 4), "train_seconds": round(train_s, 2)})
    nn_roof = {"bound": "mfma", "achieved": round(tf, 1), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "kernel": "k_nn_layer (network layers, BF16 matrix cores)",
               "launches": nl, "avg_launch_ms": round(ms / max(nl, 1), 4)}
    return out, nn_roof


def slab_schedule_cost(ctx, d, Vev, inner, tuned, method, nv_sub=4, delta=7, inner_tol=0.0):
    """The paper's region schedule on the first nv_sub eigenvectors: loops of
    the full operator for every timeslice, and loops of the slab-restricted
    operator (slab of width delta centred on every operator time) solved with
    multi-site sources and, for comparison, one operator time at a time.
    Context for the paper's cost statements (packing gain, total cost ratio);
    not part of the timed steps."""
    import torch
    T = ctx.dims[3]
    h = (delta - 1) // 2
    V4 = Vev[:, :nv_sub].contiguous()
    codes = [d.G_5]
    P = ctx.params(method=method, tol=1e-10, inner_prec=inner, rhs_block=tuned, inner_tol=inner_tol)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    (_, _, _), t_full = timed(lambda: ctx.loops_distill(V4, codes, P))
    n_full = ctx.last_solves()
    (_, _, _), t_packed = timed(lambda: ctx.loops_slab(V4, codes, delta, P))
    n_packed = ctx.last_solves()
    tau = torch.zeros((T, nv_sub, 4, nv_sub, 4), dtype=torch.complex128, device="cuda:0")

    def unpacked():
        n = 0
        for x0 in range(T):
            cut = np.zeros((4, max(ctx.dims)), dtype=np.uint8)
            cut[3, (x0 + h) % T] = 1
            cut[3, (x0 - h - 1) % T] = 1
            ctx.perambulators_tt(V4, 1 << x0, P, tau, ctx.domains(cut))
            n += ctx.last_solves()
        return n
    n_unpacked, t_unpacked = timed(unpacked)
    print("slab schedule: full %.2f s, packed %.2f s, unpacked %.2f s" % (t_full, t_packed, t_unpacked),
          file=sys.stderr, flush=True)
    return {"delta": delta, "nv": nv_sub, "full_solves": n_full, "full_s": round(t_full, 3),
            "slab_solves_packed": n_packed, "slab_packed_s": round(t_packed, 3),
            "slab_solves_unpacked": n_unpacked, "slab_unpacked_s": round(t_unpacked, 3),
            "packing_speedup": round(t_unpacked / t_packed, 2),
            "cost_ratio_full_plus_slab_over_full": round((t_full + t_packed) / t_full, 3)}


def cpu_baseline(pre, nrhs=2):
    """The oracle on the host cores: nrhs full-operator CGNR solves of the same
    workload to 1e-10 (one per spin of the source), each with its projection at
    the source timeslice."""
    import oracle
    import synth
    dims, bc = pre.dims, pre.bc
    U = synth.gauge_field(dims, pre.eps, pre.seed)
    A = oracle.clover(U, dims, pre.kappa, pre.csw)
    V = int(np.prod(dims))
    Vs = V // dims[3]
    rng = np.random.default_rng(11)
    v = rng.standard_normal((Vs, 3)) + 1j * rng.standard_normal((Vs, 3))
    v /= np.linalg.norm(v)
    its = []
    t0 = time.perf_counter()
    for a in range(nrhs):
        b = np.zeros((V, 4, 3), dtype=np.complex128)
        b[:Vs, a, :] = v
        x, it, rr = oracle.cgnr(U, A, dims, bc, pre.kappa, b, tol=1e-10)
        _ = np.einsum("xc,xbc->b", np.conj(v), x[:Vs])
        its.append(it)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the oracle's operator alone, with all threads and with one: stencil GB/s by
    # the same algorithmic-byte count as the GPU (FP64, one RHS: 1536 bytes per
    # site), and the one-thread solve rate these give at the measured CGNR
    # iterations (one D and one D^+ per iteration)
    def apply_s(reps=3):
        t = time.perf_counter()
        for _ in range(reps):
            oracle.dirac(U, A, dims, bc, pre.kappa, b)
        return (time.perf_counter() - t) / reps
    t_all = apply_s()
    old = oracle.set_threads(1)
    try:
        t_one = apply_s()
    finally:
        oracle.set_threads(old)
    bytes_apply = V * (48 * 8 + 72 * 8 + 72 * 8)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    mean_it = sum(its) / len(its)
    return {"value": nrhs / dt, "unit": "RHS/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "nproc": os.cpu_count(),
            "stencil_gbps": round(bytes_apply / t_all / 1e9, 2),
            "one_thread": {"stencil_gbps": round(bytes_apply / t_one / 1e9, 3),
                           "rhs_per_s_estimate": 1.0 / (2 * mean_it * t_one),
                           "note": "D applications timed with one OpenMP thread; the RHS rate assumes the same "
                                   "%.0f CGNR iterations (one D and one D^+ each)" % mean_it},
            "sample": "%d full-operator RHS of the %s workload: oracle FP64 CGNR to true rel. residual "
                      "1e-10 (%s iterations, %.1f s in all), each with its projection at the source timeslice; "
                      "source = one normalised Gaussian colour vector on timeslice 0, in spin %s"
                      % (nrhs, "x".join(map(str, dims)), "+".join(map(str, its)), dt,
                         " and ".join(str(a) for a in range(nrhs)))}


def production_subset(args, d, torch, synth):
    """The production shape, 32^3 x 64 (eps = 0.2, 10 APE steps, kappa = 0.127,
    csw = 1.7, Nv = 128), over four seeded ensembles (seeds 500-503), as a stated
    subset: per ensemble one packing set (timeslices 0, 16, 32, 48: one per
    temporal layer of the 8^3 x 16 domains, two per layer of the 16^3 x 32
    domains) and the first nv_sub of the 128 eigenvectors (computed on those
    four timeslices only) -- full-operator solves, packed D_Lambda solves on both
    domain sizes, loops of gamma_5, gamma_1..3 and 1 with their Gamma-tilde, and
    the full / factorised / subtracted correlators over the four ensembles at
    the separations the packing set covers (0, 16, 32, 48; per-timeslice VEV)."""
    pre = synth.PRESETS["prod_32x32x32x64"]
    dims, T, nv = pre.dims, pre.dims[3], pre.nv
    nvs = args.nv_per_step or 4
    tsel = [0, 16, 32, 48]
    tmask = sum(1 << t for t in tsel)
    codes = [d.G_5, d.G_X, d.G_Y, d.G_Z, d.G_1]
    nc = len(codes)
    loop_codes = codes + [c | d.G_TILDE for c in codes]
    inner = d.BF16 if args.inner == "bf16" else d.F32
    ctx = d.Context(dims, pre.bc, 0)
    doms = {"8x8x8x16": ctx.domains(synth.tiling_cuts(dims, (8, 8, 8, 16))),
            "16x16x16x32": ctx.domains(synth.tiling_cuts(dims, (16, 16, 16, 32)))}
    P = ctx.params(method=d.BICGSTAB_RU, tol=1e-10, inner_prec=inner, rhs_block=args.rhs_block,
                   inner_tol=args.inner_tol or 0.0)
    dev = "cuda:0"
    Vfull = torch.zeros((T, nvs, ctx.Vs, 3), dtype=torch.complex128, device=dev)
    L = {k: torch.zeros((len(loop_codes), 4, T), dtype=torch.complex128, device=dev) for k in ["full"] + list(doms)}
    solve_s = setup_s = 0.0
    logical = {k: 0 for k in L}
    packed = {k: 0 for k in L}
    secs = {k: 0.0 for k in L}
    worst = 0.0
    tuned = None
    for c, seed in enumerate(range(500, 504)):
        t0 = time.perf_counter()
        U = synth.gauge_field(dims, pre.eps, seed)
        t_gen = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.gauge_set(U)
        del U
        ctx.clover_setup(pre.kappa, pre.csw)
        ctx.ape_smear(pre.ape_steps, pre.ape_alpha)
        Vs_, lam = ctx.laplace_eigvecs_slices(nv, tsel, 1e-11)
        for k, t in enumerate(tsel):
            Vfull[t].copy_(Vs_[k, :nvs])
        del Vs_
        if tuned is None:
            tuned, _ = ctx.autotune(inner)
        torch.cuda.synchronize()
        setup_s += time.perf_counter() - t0
        print("ensemble %d: links %.1f s, set-up %.1f s (gap lambda_%d - lambda_%d = %.3g at t=0)"
              % (seed, t_gen, time.perf_counter() - t0, nv, nv - 1, lam[0, -1] - lam[0, -2]), file=sys.stderr,
              flush=True)
        for k, dom in [("full", None)] + list(doms.items()):
            tau = torch.zeros((T, nvs, 4, nvs, 4), dtype=torch.complex128, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a = ctx.perambulators_tt(Vfull, tmask, P, tau, dom)
            n_solves = ctx.last_solves()
            Lc = ctx.loops(tau, loop_codes)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            L[k][:, c].copy_(Lc)
            secs[k] += dt
            solve_s += dt
            logical[k] += 4 * nvs * len(tsel)
            packed[k] += n_solves
            worst = max(worst, a.true_rel_residual)
            print("  %s: %d solves in %.1f s, worst residual %.2e" % (k, n_solves, dt, a.true_rel_residual),
                  file=sys.stderr, flush=True)
    # correlators over the four ensembles at the covered separations
    corr = {}
    sep = [0, 16, 32, 48]
    for k in doms:
        for g, code in enumerate(codes):
            C, Cf, dC, _ = ctx.correlator(L["full"][g], L["full"][nc + g], L[k][g], L[k][nc + g], y0s=tsel,
                                          vev_mode=0)
            C, dC = C.cpu().numpy(), dC.cpu().numpy()
            name = {d.G_5: "g5", d.G_X: "g1", d.G_Y: "g2", d.G_Z: "g3", d.G_1: "1"}[code]
            corr.setdefault(name, {})["C_full"] = [[round(C[t].real, 6), round(C[t].imag, 6)] for t in sep]
            corr[name]["dC_" + k] = [[round(dC[t].real, 6), round(dC[t].imag, 6)] for t in sep]
    # the stencil of the last ensemble's full-operator solves, event-timed, every
    # launch at the block width (the tail of the queue not narrowed)
    ctx.profile_reset()
    ctx.profile_stride(1)
    ctx.set_option(d.OPT_NARROW, 0)
    ctx.profile_enable(True)
    tau = torch.zeros((T, nvs, 4, nvs, 4), dtype=torch.complex128, device=dev)
    ctx.perambulators_tt(Vfull, 1 << tsel[0], P, tau)
    ctx.profile_enable(False)
    ctx.set_option(d.OPT_NARROW, 1)
    fam = d.K_STENCIL_EO_BF16 if inner == d.BF16 else d.K_STENCIL_EO_F32
    tag = "k_dslash_eo<%s>" % ("IOBF" if inner == d.BF16 else "IO32")
    nl, ms, by = ctx.profile_get(fam)
    blk = args.rhs_block or tuned
    tile = (ctx.get_option(d.OPT_TILE_Y), ctx.get_option(d.OPT_TILE_T))
    roof = stencil_roofline(tag, nl, ms, by, ctx.V // 2, blk, traffic_key(tag, blk, "32x32x32x64", tile))
    roof["site_order_tile"] = list(tile)
    rhs = sum(logical.values())
    out = {"metric": METRIC, "value": round(rhs / solve_s, 2), "unit": "RHS/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "32x32x32x64 Wilson-clover kappa=%g csw=%g, 4 ensembles (seeds 500-503), Nv=%d "
                                  "of which the first %d per source, packing set t=0,16,32,48, domains 8^3x16 and "
                                  "16^3x32, BiCGStab %s-storage/FP32 inner with FP64 reliable updates to 1e-10"
                                  % (pre.kappa, pre.csw, nv, nvs, args.inner),
                      "lattice": "32x32x32x64", "ensembles": 4, "nv": nv, "nv_used": nvs, "timeslices": tsel,
                      "inner_tol": args.inner_tol or "library default",
                      "rhs_block": blk, "site_order_tile": list(tile)},
           "rates": {k: {"logical_rhs": logical[k], "solves": packed[k], "seconds": round(secs[k], 2),
                         "logical_rhs_per_s": round(logical[k] / secs[k], 2)} for k in L},
           "roofline": roof, "correlators_at_separations": {"separations": sep, "channels": corr},
           "worst_true_rel_residual": worst, "setup_s": round(setup_s, 1),
           "subset": "one packing set of 4 timeslices and %d of the 128 eigenvectors per ensemble: %d of the 4 x "
                     "65536 logical RHS of the full run" % (nvs, rhs)}
    print(json.dumps(out), flush=True)


def learned_form(args, d, torch, synth):
    """The learned configuration at 24^3 x 48 (kappa = 0.126, csw = 1.6), as a
    stated subset of its training: the network is trained on (residual, error)
    pairs the solver generates, streamed from the eight training ensembles
    (seeds 100-107; each ensemble's pairs are generated, trained on and
    discarded before the next), then judged on a held-out ensemble (seed 200):
    FGMRES(16) with the trained network and without the FP64 fallback, the
    same with the untrained network (the gain), unpreconditioned FP64
    BiCGStab, plain FP64 CGNR and the mixed-precision batched solver, all to
    true relative residual 1e-10 on the same 8 sources (Gaussian colour vectors
    on timeslice 0, two vectors x four spins)."""
    pre = synth.PRESETS["batch_24x24x24x48"]
    dims = pre.dims
    npairs, steps = args.nn_pairs, args.nn_steps
    ctx = d.Context(dims, pre.bc, 0)
    ctx.gauge_set(synth.gauge_field(dims, pre.eps, 100))
    ctx.clover_setup(pre.kappa, pre.csw)
    net = d.Net(ctx, 16, 7)
    untrained = d.Net(ctx, 16, 7)
    train = []
    t0 = time.perf_counter()
    for seed in range(100, 108):
        if seed != 100:
            ctx.gauge_set(synth.gauge_field(dims, pre.eps, seed))
            ctx.clover_setup(pre.kappa, pre.csw)
            net.refresh()
        ts = net.train(npairs, snap_iters=(0, 16, 64, 192), batch=4, steps=steps, lr=2e-3, seed=seed)
        train.append({"seed": seed, "pairs": ts.pairs, "steps": ts.steps, "loss_first": round(ts.first_loss, 4),
                      "loss_final": round(ts.final_loss, 4), "gen_s": round(ts.gen_seconds, 1),
                      "train_s": round(ts.train_seconds, 1)})
        print("trained on seed %d: loss %.3f -> %.3f" % (seed, ts.first_loss, ts.final_loss), file=sys.stderr,
              flush=True)
    train_s = time.perf_counter() - t0
    ctx.gauge_set(synth.gauge_field(dims, pre.eps, 200))
    ctx.clover_setup(pre.kappa, pre.csw)
    net.refresh()
    untrained.refresh()
    Vn = synth.random_colour_vectors(dims[3], 2, ctx.Vs, 201)
    b = torch.zeros((8, ctx.V, 4, 3), dtype=torch.complex128, device="cuda:0")
    for i in range(2):
        for a in range(4):
            b[4 * i + a, :ctx.Vs, a, :] = torch.from_numpy(Vn[0, i]).to("cuda:0")
    out = {}

    def run(name, P, nb, allow=False):
        bb = b[:nb].contiguous()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = ctx.solve_multi_rhs(bb, P, allow_noconv=allow)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[name] = {"rhs_per_s": round(nb / dt, 3), "rhs": nb, "iters": max(s.iters for s in st),
                     "converged": all(s.converged for s in st), "fallback_used": max(s.fallback_used for s in st),
                     "worst_true_rel_residual": max(s.true_rel_residual for s in st)}
        print("%s: %.3f RHS/s, %d iterations" % (name, nb / dt, out[name]["iters"]), file=sys.stderr, flush=True)

    ctx.profile_reset()
    ctx.profile_stride(1)
    ctx.profile_enable(True)
    run("fgmres16_trained_network_no_fallback",
        ctx.params(method=d.FGMRES_NN, tol=1e-10, net=net, restart=16, rhs_block=8, fallback=0, max_iter=1500), 8,
        True)
    ctx.profile_enable(False)
    nl, ms, fl = ctx.profile_get(d.K_NN)
    tf = fl / (ms / 1e3) / 1e12 if ms > 0 else 0.0
    run("fgmres16_untrained_network_no_fallback",
        ctx.params(method=d.FGMRES_NN, tol=1e-10, net=untrained, restart=16, rhs_block=8, fallback=0, max_iter=800),
        8, True)
    ctx.set_option(d.OPT_EO, 0)
    run("bicgstab_f64_unpreconditioned", ctx.params(method=d.BICGSTAB_DC, tol=1e-10, inner_prec=d.F64,
                                                    rhs_block=1), 2)
    ctx.set_option(d.OPT_EO, 1)
    run("cgnr_f64_plain", ctx.params(method=d.CGNR_F64, tol=1e-10, rhs_block=1), 2)
    run("mixed_batched_reliable_updates_no_network", ctx.params(method=d.BICGSTAB_RU, tol=1e-10, inner_prec=d.BF16,
                                                                 rhs_block=8), 8)
    res = {"metric": "learned preconditioner at 24x24x24x48: RHS/s and iterations at true rel. residual 1e-10",
           "workload": "24x24x24x48 kappa=%g csw=%g; network 16 channels, 3^4 parallel-transport kernels; trained on "
                       "%d pairs per ensemble streamed from seeds 100-107 (%d in all), %d Adam steps each; judged on "
                       "seed 200" % (pre.kappa, pre.csw, npairs, 8 * npairs, steps),
           "training": train, "training_s": round(train_s, 1), "solvers": out,
           "nn_roofline": {"bound": "mfma", "achieved": round(tf, 1), "peak": MFMA_BF16_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "launches": nl,
                           "avg_launch_ms": round(ms / max(nl, 1), 3)}}
    print(json.dumps(res), flush=True)


def main():
    t_start = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", choices=["bf16", "f32"], default="bf16")
    ap.add_argument("--rhs-block", type=int, default=0)
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="reliable-update threshold delta (0 = library default; default 0.1 for BF16 reliable "
                         "updates on 24^3x48, the library default elsewhere)")
    ap.add_argument("--method", choices=["ru", "dc"], default="ru",
                    help="BiCGStab with reliable updates (default) or inside FP64 defect correction")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the solver comparison and the region-schedule legs after the timed steps")
    ap.add_argument("--nv-per-step", type=int, default=0,
                    help="eigenvectors per step (a divisor of Nv; default Nv/4 at 24^3x48, Nv at 16^3x32)")
    ap.add_argument("--workload", choices=["batch_24x24x24x48", "prec_16x16x16x32", "prod_32x32x32x64",
                                           "learned_24x24x24x48"], default="batch_24x24x24x48")
    ap.add_argument("--nn-pairs", type=int, default=64, help="learned workload: pairs per training ensemble")
    ap.add_argument("--nn-steps", type=int, default=150, help="learned workload: Adam steps per training ensemble")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solves of different right-hand sides are independent, so "
              "the path shards by right-hand side without exchange (see the design notes); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2609_37049_amd as d

    torch.cuda.set_device(0)
    if args.workload == "prod_32x32x32x64":
        production_subset(args, d, torch, synth)
        return
    if args.workload == "learned_24x24x24x48":
        learned_form(args, d, torch, synth)
        return
    pre = synth.PRESETS[args.workload]
    dims = pre.dims
    T = dims[3]
    codes = [d.G_1, d.G_5, d.G_X, d.G_Y, d.G_Z]
    nc = len(codes)
    loop_codes = codes + [c | d.G_TILDE for c in codes]   # Gamma and Gamma~ = g4 Gamma^+ g4, from the library
    torch.cuda.set_device(0)
    U = synth.gauge_field(dims, pre.eps, pre.seed)
    ctx = d.Context(dims, pre.bc, 0)
    cut = synth.tiling_cuts(dims, pre.block)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.gauge_set(U)
    ctx.clover_setup(pre.kappa, pre.csw)
    ctx.ape_smear(pre.ape_steps, pre.ape_alpha)
    Vev, lam = ctx.laplace_eigvecs(pre.nv, 1e-11)
    dom = ctx.domains(cut)
    inner = d.BF16 if args.inner == "bf16" else d.F32
    tuned, tune_cost = ctx.autotune(inner)
    nv = pre.nv
    nvs = args.nv_per_step or (nv // 4 if args.workload == "batch_24x24x24x48" else nv)
    if nv % nvs:
        raise SystemExit("--nv-per-step must divide Nv = %d" % nv)
    nq = nv // nvs
    # the eigenvector groups of the steps, each [T][nvs][Vs][3] (resident before timing)
    Vq = [Vev[:, q * nvs:(q + 1) * nvs].contiguous() for q in range(nq)]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print("set-up done in %.1f s (rhs block %d)" % (setup_s, tuned), file=sys.stderr, flush=True)

    method = d.BICGSTAB_RU if args.method == "ru" else d.BICGSTAB_DC
    # the reliable-update threshold delta of the full-operator solves: 0.1 for
    # BF16 on the 24^3x48 batching shape, where it was swept (3e-2, the library
    # default, is best at 16^3x32 and for the faster-converging D_Lambda solves)
    inner_tol = args.inner_tol
    if inner_tol is None:
        inner_tol = 0.1 if (args.workload == "batch_24x24x24x48" and args.inner == "bf16" and args.method == "ru") \
            else 0.0
    P = ctx.params(method=method, tol=1e-10, inner_prec=inner, rhs_block=args.rhs_block, inner_tol=inner_tol)
    P_blk = ctx.params(method=method, tol=1e-10, inner_prec=inner, rhs_block=args.rhs_block,
                       inner_tol=args.inner_tol or 0.0)
    dev = "cuda:0"
    # perambulators tau(t,t) per eigenvector group, filled set by set
    tau_f = [torch.zeros((T, nvs, 4, nvs, 4), dtype=torch.complex128, device=dev) for _ in range(nq)]
    tau_b = [torch.zeros_like(tau_f[0]) for _ in range(nq)]
    layer = pre.block[3]
    groups = [sum(1 << (g + layer * k) for k in range(T // layer)) for g in range(layer)]
    combos = [(g, q) for g in range(len(groups)) for q in range(nq)]

    def step(k):
        g, q = combos[k % len(combos)]
        msk = groups[g]
        ta = time.perf_counter()
        a1 = ctx.perambulators_tt(Vq[q], msk, P, tau_f[q])
        n_full = ctx.last_solves()
        tb = time.perf_counter()
        a2 = ctx.perambulators_tt(Vq[q], msk, P_blk, tau_b[q], dom)
        n_blk = ctx.last_solves()
        tc = time.perf_counter()
        # partial loops over this group's eigenvectors, for the Gamma's and their
        # Gamma~'s, and the full / factorised / subtracted correlators of them
        Lf = ctx.loops(tau_f[q], loop_codes)
        Lb = ctx.loops(tau_b[q], loop_codes)
        for c in range(nc):
            ctx.correlator(Lf[c:c + 1], Lf[nc + c:nc + c + 1], Lb[c:c + 1], Lb[nc + c:nc + c + 1])
        torch.cuda.synchronize()
        logical = 4 * nvs * bin(msk).count("1")
        return (logical, n_full, n_blk, max(a1.true_rel_residual, a2.true_rel_residual), a1, a2,
                tb - ta, tc - tb)

    for k in range(args.warmup):
        step(k)
        print("warmup step %d done" % k, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rhs_full = rhs_blk = solves_full = solves_blk = 0
    t_full = t_blk = 0.0
    worst = 0.0
    iters = 0
    for k in range(args.warmup, args.warmup + args.steps):
        logical, nf, nb, res, a1, a2, dtf, dtb = step(k)
        rhs_full += logical
        rhs_blk += logical
        solves_full += nf
        solves_blk += nb
        t_full += dtf
        t_blk += dtb
        worst = max(worst, res)
        iters += a1.iters + a2.iters
        print("timed step %d: %d logical RHS, %d solves, worst residual %.2e" % (k, 2 * logical, nf + nb, res),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rhs = rhs_full + rhs_blk
    # The production steps above run their inner iterations as HIP graphs; the
    # per-launch stencil times come from one more pass of a step's full-operator
    # solves (the dominant launches: the unmasked stencil; the D_Lambda solves use
    # the masked instance) with every stencil launch bracketed by HIP events on
    # the context stream (eager launches), and its projections.  The queue's
    # tail is not narrowed in this pass, so that every timed launch has the
    # block width the roofline entry names.
    ctx.profile_reset()
    ctx.profile_stride(1)
    ctx.set_option(d.OPT_NARROW, 0)
    ctx.profile_enable(True)
    g_next, q_next = combos[(args.warmup + args.steps) % len(combos)]
    ctx.perambulators_tt(Vq[q_next], groups[g_next], P, tau_f[q_next])
    ctx.profile_enable(False)
    ctx.set_option(d.OPT_NARROW, 1)
    # dominant kernel: the inner-precision stencil family with the most launches
    # (the even-odd half-lattice stencil when every extent is even)
    fams = {"k_dslash<%s>" % io: fam for io, fam in (("IOBF", d.K_STENCIL_BF16), ("IO32", d.K_STENCIL_F32))}
    fams.update({"k_dslash_eo<%s>" % io: fam for io, fam in (("IOBF", d.K_STENCIL_EO_BF16),
                                                              ("IO32", d.K_STENCIL_EO_F32))})
    io = "IOBF" if inner == d.BF16 else "IO32"
    cands = [t for t in fams if io in t]
    stats = {t: ctx.profile_get(fams[t]) for t in cands}
    kernel_tag = max(stats, key=lambda t: stats[t][0])
    nl, ms, by = stats[kernel_tag]
    ml, mms, mfl = ctx.profile_get(d.K_MFMA)
    mtf = mfl / (mms / 1e3) / 1e12 if mms > 0 else 0.0
    mfma_roof = {"bound": "mfma", "achieved": round(mtf, 2), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": round(mtf / FP64_MFMA_PEAK_TFLOPS, 4),
                 "kernel": "k_zgemm_hn (perambulator projection V(t)^+ X(t), FP64 matrix cores)",
                 "launches": ml, "avg_launch_ms": round(mms / max(ml, 1), 4),
                 "flop_per_launch": round(mfl / max(ml, 1))}
    sites = ctx.V // 2 if "_eo" in kernel_tag else ctx.V
    print("profiled step done: %d launches of %s" % (nl, kernel_tag), file=sys.stderr, flush=True)
    blk = args.rhs_block or tuned
    lat = "x".join(map(str, dims))
    big = args.workload != "prec_16x16x16x32"
    tile = (ctx.get_option(d.OPT_TILE_Y), ctx.get_option(d.OPT_TILE_T))
    roof = stencil_roofline(kernel_tag, nl, ms, by, sites, blk, traffic_key(kernel_tag, blk, lat, tile))
    roof["site_order_tile"] = list(tile)
    comparison = nn_roof = slab = None
    if not args.no_legs:
        comparison, nn_roof = solver_comparison(ctx, d, Vev, inner, args.rhs_block or tuned, T, inner_tol)
        slab = slab_schedule_cost(ctx, d, Vev, inner, args.rhs_block or tuned, method, nv_sub=2 if big else 4,
                                  inner_tol=inner_tol)
    # the stencil at the batching shape when the workload is the smaller one
    large = None if (args.no_legs or big) else stencil_at_batch_shape(d, inner, blk)
    if large:
        print("24^3x48 stencil: %.1f GB/s over %d launches" % (large["achieved"], large["launches_timed"]),
              file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": round(rhs / dt, 2), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s Wilson-clover kappa=%g csw=%g, Nv=%d (%d per step), domains %s, "
                               "BiCGStab %s-storage/FP32 inner, %s, to FP64 true residual 1e-10" % (
                                   lat, pre.kappa, pre.csw, nv, nvs, "x".join(map(str, pre.block)),
                                   args.inner, "reliable updates" if args.method == "ru" else "FP64 defect correction"),
                   "lattice": lat, "kappa": pre.kappa, "csw": pre.csw, "nv": nv, "nv_per_step": nvs,
                   "domains": "x".join(map(str, pre.block)), "rhs_block": args.rhs_block or tuned,
                   "site_order_tile": {"y_rows": ctx.get_option(d.OPT_TILE_Y),
                                       "timeslices": ctx.get_option(d.OPT_TILE_T)},
                   "autotune_us_per_rhs_iter": {str(k): round(v, 3) for k, v in tune_cost.items()},
                   "inner_storage": args.inner, "hip_graphs": True, "method": args.method,
                   "inner_tol": {"full_operator": inner_tol if inner_tol > 0 else "library default",
                                 "d_lambda": args.inner_tol or "library default"},
                   "outer": "f64", "logical_rhs_per_step": rhs // max(args.steps, 1),
                   "solves_per_step": (solves_full + solves_blk) // max(args.steps, 1),
                   "step": "one packing set (%d timeslices, one per temporal layer) x %d eigenvectors x 4 spins: "
                           "sources, full-operator solves, packed D_Lambda solves, projections, loops of 5 "
                           "Gamma and their Gamma-tilde, full/factorised/subtracted correlators"
                           % (T // layer, nvs)},
        "rates": {"full_operator_rhs_per_s": round(rhs_full / t_full, 2) if t_full > 0 else None,
                  "d_lambda_logical_rhs_per_s": round(rhs_blk / t_blk, 2) if t_blk > 0 else None,
                  "d_lambda_packed_solves_per_s": round(solves_blk / t_blk, 2) if t_blk > 0 else None,
                  "full_operator_s": round(t_full, 3), "d_lambda_s": round(t_blk, 3),
                  "note": "value counts each packed D_Lambda solve as the %d logical right-hand sides it carries"
                          % (T // layer)},
        "roofline": roof,
        "roofline_24x24x24x48": large,
        "solver_comparison": comparison,
        "nn_roofline": nn_roof,
        "perambulator_roofline": mfma_roof,
        "slab_schedule": slab,
        "worst_true_rel_residual": worst,
        "inner_iterations": iters,
        "setup_s": round(setup_s, 3),
    }
    if not args.no_cpu_baseline:
        # about 15 s of host work at 16^3x32; one RHS (about 60 s) at 24^3x48
        out["cpu_baseline"] = cpu_baseline(pre, 1 if big else 2)
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
