"""GPU parity of the solvers: FP64 CGNR, BiCGStab with FP32/BF16 inner
solves inside FP64 defect correction, and BiCGStab with reliable updates,
full and domain-restricted operators.
Judged by the oracle: its own solution on small lattices, and the true
residual computed with the oracle's operator at the full workload size."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    import paper_2609_37049_amd as d
    d.lib()
    return d


@pytest.fixture(scope="module")
def plain(disco):
    pre = synth.PRESETS["plain_4x4x4x4"]
    U = synth.gauge_field(pre.dims, pre.eps, pre.seed)
    ctx = disco.Context(pre.dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(pre.kappa, pre.csw)
    A = oracle.clover(U, pre.dims, pre.kappa, pre.csw)
    return pre, ctx, U, A


def _true_rel_res(U, A, dims, kappa, b, x, cut=None):
    r = b - oracle.dirac(U, A, dims, BC, kappa, x, cut=cut)
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=(1, 2, 3)) / np.sum(np.abs(b) ** 2, axis=(1, 2, 3)))


@pytest.mark.parametrize("method,inner", [("CGNR_F64", "F64"), ("BICGSTAB_DC", "F32"), ("BICGSTAB_DC", "BF16"),
                                          ("BICGSTAB_DC", "F64"), ("BICGSTAB_RU", "F32"), ("BICGSTAB_RU", "BF16")])
@pytest.mark.parametrize("blocked", [False, True])
def test_solver_matches_oracle_small(disco, plain, method, inner, blocked):
    pre, ctx, U, A = plain
    _say("solve", method, inner, blocked)
    dims = pre.dims
    V = int(np.prod(dims))
    cut = synth.tiling_cuts(dims, pre.block) if blocked else None
    dom = ctx.domains(cut) if blocked else None
    b = synth.random_spinor(V, 5, 31)
    tol = 1e-12
    P = ctx.params(method=getattr(disco, method), tol=tol, inner_prec=getattr(disco, inner), rhs_block=4)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P, dom)
    x = x.cpu().numpy()
    rr = _true_rel_res(U, A, dims, pre.kappa, b, x, cut)
    assert rr.max() <= tol * 1.01, rr
    assert all(s.converged for s in st)
    # both are evaluations of the same residual; below ~1e-14 FP64 rounding of b - D x dominates
    rep = [s.true_rel_residual for s in st]
    assert all(abs(a - r) <= max(1e-2 * r, 2e-15) for a, r in zip(rep, rr)), (rep, list(rr))
    xo, _, _ = oracle.cgnr(U, A, dims, BC, pre.kappa, b[2], cut=cut, tol=1e-13)
    assert np.abs(x[2] - xo).max() / np.abs(xo).max() < 1e-10


def test_solver_zero_rhs_and_empty(disco, plain):
    pre, ctx, U, A = plain
    V = int(np.prod(pre.dims))
    b = np.zeros((2, V, 4, 3), dtype=np.complex128)
    b[1] = synth.random_spinor(V, 1, 3)[0]
    P = ctx.params(tol=1e-11)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P)
    x = x.cpu().numpy()
    assert np.abs(x[0]).max() == 0
    assert st[1].true_rel_residual <= 1e-11
    x, st = ctx.solve_multi_rhs(ctx.dev(b[:0]), P)
    assert x.shape[0] == 0


def test_solver_reports_noconv(disco, plain):
    pre, ctx, U, A = plain
    V = int(np.prod(pre.dims))
    b = synth.random_spinor(V, 2, 5)
    P = ctx.params(method=disco.CGNR_F64, tol=1e-12, max_iter=3)
    with pytest.raises(disco.DiscoError) as e:
        ctx.solve_multi_rhs(ctx.dev(b), P)
    assert e.value.code == disco.ENOCONV
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P, allow_noconv=True)
    assert not st[0].converged and st[0].true_rel_residual > 1e-12


def test_batched_equals_unbatched(disco, plain):
    pre, ctx, U, A = plain
    V = int(np.prod(pre.dims))
    b = synth.random_spinor(V, 8, 41)
    out = {}
    for blk in (1, 2, 8):
        P = ctx.params(tol=1e-12, rhs_block=blk)
        out[blk] = ctx.solve_multi_rhs(ctx.dev(b), P)[0].cpu().numpy()
    for blk in (1, 2):
        assert np.abs(out[blk] - out[8]).max() / np.abs(out[8]).max() < 1e-10


def test_full_size_mixed_precision_solve(disco):
    """16^3 x 32 mixed-precision workload: FP32 and BF16 inner BiCGStab with
    FP64 defect correction and with reliable updates to 1e-10, full and block
    operator; the true
    residual is recomputed with the oracle's FP64 operator."""
    pre = synth.PRESETS["prec_16x16x16x32"]
    dims = pre.dims
    _say("full-size solve", dims)
    U = synth.gauge_field(dims, pre.eps, pre.seed)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(pre.kappa, pre.csw)
    A = oracle.clover(U, dims, pre.kappa, pre.csw)
    V = int(np.prod(dims))
    cut = synth.tiling_cuts(dims, pre.block)
    dom = ctx.domains(cut)
    b = synth.random_spinor(V, 16, 55)
    for method, inner in ((disco.BICGSTAB_DC, disco.F32), (disco.BICGSTAB_DC, disco.BF16),
                          (disco.BICGSTAB_RU, disco.F32), (disco.BICGSTAB_RU, disco.BF16)):
        for d, c in ((None, None), (dom, cut)):
            _say("  method", method, "inner", inner, "block" if d else "full")
            P = ctx.params(method=method, tol=1e-10, inner_prec=inner, rhs_block=16)
            x, st = ctx.solve_multi_rhs(ctx.dev(b), P, d)
            x = x.cpu().numpy()
            rr = _true_rel_res(U, A, dims, pre.kappa, b[:3], x[:3], c)
            assert rr.max() <= 1e-10 * 1.01, rr
            assert all(s.converged for s in st)


def test_graph_replays_equal_eager(disco):
    """Inner iterations captured as HIP graphs give bitwise the same solutions
    as eager launches: the chunk graph is replayed many times per solve, with
    host reads and FP64 outer-residual work between replays."""
    pre = synth.PRESETS["plain_4x4x4x4"]
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.3, 21)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(0.125, 1.3)
    V = int(np.prod(dims))
    b = ctx.dev(synth.random_spinor(V, 24, 22))
    out = {}
    # (method, inner precision, lanes): 3 lanes refill from the queue of 24
    cases = [(m, i, 8) for m in (disco.BICGSTAB_DC, disco.BICGSTAB_RU) for i in (disco.F32, disco.BF16)]
    cases += [(disco.BICGSTAB_RU, disco.BF16, 3)]
    for g in (0, 1):
        ctx.set_option(disco.OPT_GRAPHS, g)
        for m, inner, blk in cases:
            P = ctx.params(method=m, tol=1e-11, inner_prec=inner, rhs_block=blk, check_every=5)
            x, st = ctx.solve_multi_rhs(b, P)
            out[(g, m, inner, blk)] = (x.cpu().numpy(), [s.iters for s in st], [s.outer_iters for s in st])
    for key in cases:
        assert out[(0,) + key][1:] == out[(1,) + key][1:]
        assert np.array_equal(out[(0,) + key][0], out[(1,) + key][0])
    ctx.set_option(disco.OPT_GRAPHS, 1)


def test_stage_option_same_operator(disco):
    dims = (8, 8, 4, 8)
    U = synth.gauge_field(dims, 0.3, 23)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(0.12, 1.1)
    V = int(np.prod(dims))
    psi = synth.random_spinor(V, 16, 24)
    res = {}
    for stage in (0, 1):
        ctx.set_option(disco.OPT_STAGE, stage)
        res[stage] = ctx.dirac_apply(ctx.dev(psi), disco.F32).cpu().numpy()
    ctx.set_option(disco.OPT_STAGE, -1)
    assert np.array_equal(res[0], res[1])


def test_autotune_picks_a_block(disco):
    dims = (8, 8, 8, 16)
    U = synth.gauge_field(dims, 0.25, 25)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(0.125, 1.5)
    best, cost = ctx.autotune(disco.BF16)
    assert best in (8, 16, 32, 64)
    assert all(c > 0 for c in cost.values()) and cost[best] == min(cost.values())
    V = int(np.prod(dims))
    b = synth.random_spinor(V, 5, 26)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), ctx.params(tol=1e-10, inner_prec=disco.BF16, rhs_block=0))
    A = oracle.clover(U, dims, 0.125, 1.5)
    assert _true_rel_res(U, A, dims, 0.125, b, x.cpu().numpy()).max() <= 1e-10 * 1.01


@pytest.mark.parametrize("inner", ["F32", "BF16", "F64"])
@pytest.mark.parametrize("blocked", [False, True])
def test_even_odd_inner_solves(disco, inner, blocked):
    """Inner BiCGStab on the even-odd Schur complement against the same solver
    on the full operator: both judged by the oracle's FP64 true residual of
    the full (or domain-restricted) system; the Schur form needs fewer inner
    iterations and no fallback."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.124, 1.2
    U = synth.gauge_field(dims, 0.3, 51)
    A = oracle.clover(U, dims, kappa, csw)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, csw)
    cut = synth.tiling_cuts(dims, (4, 4, 4, 4)) if blocked else None
    dom = ctx.domains(cut) if blocked else None
    b = synth.random_spinor(ctx.V, 4, 52)
    tol = 1e-12 if inner != "BF16" else 1e-10
    iters = {}
    for eo in (1, 0):
        ctx.set_option(disco.OPT_EO, eo)
        P = ctx.params(method=disco.BICGSTAB_DC, tol=tol, inner_prec=getattr(disco, inner), rhs_block=4)
        x, st = ctx.solve_multi_rhs(ctx.dev(b), P, dom)
        rr = _true_rel_res(U, A, dims, kappa, b, x.cpu().numpy(), cut)
        _say("  even-odd %d inner %s blocked %s: %d inner iterations, %d cycles, oracle residual %.2e" %
             (eo, inner, blocked, st[0].iters, st[0].outer_iters, rr.max()))
        assert all(s.fallback_used == 0 for s in st)
        assert rr.max() <= tol * 1.05
        for k in range(4):
            assert abs(rr[k] - st[k].true_rel_residual) <= max(1e-2 * rr[k], 2e-15)
        iters[eo] = st[0].iters
    ctx.set_option(disco.OPT_EO, 1)
    assert iters[1] <= iters[0]


@pytest.mark.parametrize("inner", ["F32", "BF16"])
@pytest.mark.parametrize("eo", [1, 0])
@pytest.mark.parametrize("blocked", [False, True])
def test_reliable_updates(disco, inner, eo, blocked):
    """BiCGStab with reliable updates, on the even-odd Schur complement and on
    the full operator, full and domain-restricted: every right-hand side meets
    the tolerance by the oracle's FP64 true residual, without the fallback,
    with the residual the library reports; a zero right-hand side stays zero."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.124, 1.2
    U = synth.gauge_field(dims, 0.3, 61)
    A = oracle.clover(U, dims, kappa, csw)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, csw)
    ctx.set_option(disco.OPT_EO, eo)
    cut = synth.tiling_cuts(dims, (4, 4, 4, 4)) if blocked else None
    dom = ctx.domains(cut) if blocked else None
    b = synth.random_spinor(ctx.V, 6, 62)
    b[3] = 0
    tol = 1e-12 if inner == "F32" else 1e-10
    P = ctx.params(method=disco.BICGSTAB_RU, tol=tol, inner_prec=getattr(disco, inner), rhs_block=6)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P, dom)
    ctx.set_option(disco.OPT_EO, 1)
    x = x.cpu().numpy()
    assert np.abs(x[3]).max() == 0
    live = [0, 1, 2, 4, 5]
    rr = _true_rel_res(U, A, dims, kappa, b[live], x[live], cut)
    _say("  reliable updates %s eo %d blocked %s: %d iterations, %d updates, oracle residual %.2e" %
         (inner, eo, blocked, st[0].iters, st[0].outer_iters, rr.max()))
    assert all(s.fallback_used == 0 for s in st)
    assert rr.max() <= tol * 1.05
    for k, i in enumerate(live):
        assert abs(rr[k] - st[i].true_rel_residual) <= max(1e-2 * rr[k], 2e-15)


def test_reliable_updates_fallback_and_errors(disco, plain):
    """An iteration cap below what the inner process needs hands over to the
    FP64 CGNR fallback, which reports its result truthfully; FP64 storage is
    not a reliable-update precision."""
    pre, ctx, U, A = plain
    V = int(np.prod(pre.dims))
    b = synth.random_spinor(V, 3, 63)
    P = ctx.params(method=disco.BICGSTAB_RU, tol=1e-12, inner_prec=disco.BF16, max_iter=6, rhs_block=3)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P, allow_noconv=True)
    assert all(s.fallback_used == 1 for s in st)
    rr = _true_rel_res(U, A, pre.dims, pre.kappa, b, x.cpu().numpy())
    for k in range(3):
        assert abs(rr[k] - st[k].true_rel_residual) <= max(1e-2 * rr[k], 2e-15)
        assert st[k].converged == (rr[k] <= 1e-12 * 1.01)
    with pytest.raises(disco.DiscoError) as e:
        ctx.solve_multi_rhs(ctx.dev(b), ctx.params(method=disco.BICGSTAB_RU, tol=1e-10, inner_prec=disco.F64))
    assert e.value.code == disco.EINVAL


@pytest.mark.parametrize("inner", ["F32", "BF16"])
def test_reliable_updates_lane_refill(disco, inner):
    """Eleven right-hand sides (four of them zero) through 3 lanes: a lane whose
    right-hand side converges takes the next one at that update.  Every solution
    meets the tolerance by the oracle's FP64 residual, with the residual the
    library reports, and matches the solution of an 11-lane block (no refill) to
    the accuracy both solves reach; zero right-hand sides give x = 0."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.124, 1.2
    U = synth.gauge_field(dims, 0.3, 71)
    A = oracle.clover(U, dims, kappa, csw)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, csw)
    b = synth.random_spinor(ctx.V, 11, 72)
    b[4] = 0
    b[8:] = 0  # zero right-hand sides finish at once, also at the end of the queue
    b[7] *= 1e-3  # a differently scaled right-hand side
    tol = 1e-12 if inner == "F32" else 1e-10
    sol = {}
    for blk in (3, 11):
        P = ctx.params(method=disco.BICGSTAB_RU, tol=tol, inner_prec=getattr(disco, inner), rhs_block=blk)
        x, st = ctx.solve_multi_rhs(ctx.dev(b), P)
        x = x.cpu().numpy()
        sol[blk] = x
        for k in (4, 8, 9, 10):
            assert np.abs(x[k]).max() == 0
        live = [k for k in range(11) if k not in (4, 8, 9, 10)]
        rr = _true_rel_res(U, A, dims, kappa, b[live], x[live])
        _say("  refill %s block %d: iterations per rhs %s, oracle residual %.2e" %
             (inner, blk, [s.iters for s in st], rr.max()))
        assert rr.max() <= tol * 1.05
        assert all(s.fallback_used == 0 and s.converged for s in st)
        for q, k in enumerate(live):
            assert abs(rr[q] - st[k].true_rel_residual) <= max(1e-2 * rr[q], 2e-15)
    for k in range(11):
        if k in (4, 8, 9, 10):
            continue
        d = np.linalg.norm(sol[3][k] - sol[11][k]) / np.linalg.norm(sol[11][k])
        assert d < 1e4 * tol, (k, d)  # a lane mix-up would show at O(1)


@pytest.mark.parametrize("fallback", [1, 0])
def test_reliable_updates_queue_survives_the_fallback(disco, fallback):
    """Eleven right-hand sides through 3 lanes with an inner iteration cap far
    below what a solve needs, so the first wave stops early.  The lanes in
    flight go to the FP64 fallback (or, without it, come back unconverged), and
    the rest of the queue runs on in a fresh Krylov process instead of coming
    back as x = 0: with the fallback every right-hand side meets the tolerance
    by the oracle's FP64 residual; without it every one has been worked on and
    reports its true residual."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.124, 1.2
    U = synth.gauge_field(dims, 0.3, 73)
    A = oracle.clover(U, dims, kappa, csw)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, csw)
    b = synth.random_spinor(ctx.V, 11, 74)
    tol = 1e-10
    P = ctx.params(method=disco.BICGSTAB_RU, tol=tol, inner_prec=disco.BF16, rhs_block=3, max_iter=4,
                   fallback=fallback)
    x, st = ctx.solve_multi_rhs(ctx.dev(b), P, allow_noconv=True)
    x = x.cpu().numpy()
    rr = _true_rel_res(U, A, dims, kappa, b, x)
    _say("  queue with fallback=%d: residuals %s, fallback %s" %
         (fallback, ["%.1e" % r for r in rr], [s.fallback_used for s in st]))
    for k in range(11):
        assert abs(rr[k] - st[k].true_rel_residual) <= max(1e-2 * rr[k], 2e-15)
        assert st[k].iters > 0
    if fallback:
        assert rr.max() <= tol * 1.05
        assert all(s.converged and s.fallback_used == 1 for s in st)
    else:
        assert rr.max() < 0.9          # every one was worked on, none returned as x = 0
        assert all(s.fallback_used == 0 for s in st)
        assert all(s.converged == (r <= tol) for s, r in zip(st, rr))


@pytest.mark.parametrize("inner", ["F32", "BF16"])
def test_reliable_updates_narrow_the_tail(disco, capfd, inner):
    """Forty right-hand sides (two of them zero, one scaled by 1e-3) through a
    block of 32 lanes: once the queue is empty and at most half of the lanes
    are open, the open ones move into a block of 16 and go on from their
    current iterates.  Every solution meets the tolerance by the oracle's FP64
    residual, the library reports that residual and the iterations each right-
    hand side took over both blocks, and the solutions agree with a run that
    keeps the width (a lane mix-up in the move would show at O(1))."""
    import os
    dims = (8, 8, 8, 8)
    kappa, csw = 0.124, 1.2
    U = synth.gauge_field(dims, 0.3, 81)
    A = oracle.clover(U, dims, kappa, csw)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, csw)
    b = synth.random_spinor(ctx.V, 40, 82)
    b[5] = 0
    b[39] = 0
    b[33] *= 1e-3
    tol = 1e-12 if inner == "F32" else 1e-10
    live = [k for k in range(40) if k not in (5, 39)]
    sol = {}
    for narrow in (1, 0):
        ctx.set_option(disco.OPT_NARROW, narrow)
        P = ctx.params(method=disco.BICGSTAB_RU, tol=tol, inner_prec=getattr(disco, inner), rhs_block=32)
        os.environ["DISCO_TRACE"] = "1"
        try:
            x, st = ctx.solve_multi_rhs(ctx.dev(b), P)
        finally:
            del os.environ["DISCO_TRACE"]
        moves = capfd.readouterr().err.count("move into a block of 16")
        x = x.cpu().numpy()
        sol[narrow] = x
        assert np.abs(x[5]).max() == 0 and np.abs(x[39]).max() == 0
        rr = _true_rel_res(U, A, dims, kappa, b[live], x[live])
        _say("  narrow=%d %s: %d moves, iterations per rhs %s, oracle residual %.2e" %
             (narrow, inner, moves, [s.iters for s in st], rr.max()))
        assert moves == (1 if narrow else 0)
        assert rr.max() <= tol * 1.05
        assert all(s.fallback_used == 0 and s.converged for s in st)
        assert all(st[k].iters > 0 for k in live)
        for q, k in enumerate(live):
            assert abs(rr[q] - st[k].true_rel_residual) <= max(1e-2 * rr[q], 2e-15)
    ctx.set_option(disco.OPT_NARROW, 1)
    for k in live:
        d = np.linalg.norm(sol[1][k] - sol[0][k]) / np.linalg.norm(sol[0][k])
        assert d < 1e4 * tol, (k, d)
