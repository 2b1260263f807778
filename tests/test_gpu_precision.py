"""The error of the production precision form against the FP64 oracle, per loop
and per correlator timeslice.

The production solver stores its inner vectors in BF16 and computes in FP32
(BiCGStab on the even-odd Schur complement, 64-wide blocks fed from one
queue), with FP64 reliable updates against the FP64 true residual.  Its error
in the loops and correlators comes only from where it stops: both sides take
the same smearing vectors, the GPU solves to true relative residual 1e-12 and
the oracle (FP64 CGNR) to 1e-13.  The bars are those of the plain method:
loops to relative 1e-10 per channel (max over t of |dL| / max over t of
|L_ref|), correlators to 1e-10 of max |C_ref| plus the FP64 rounding floor of
the VEV-subtracted products (64 eps max|L|^2).  The tables the tests print
are the measured errors.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
CODES = [0, 1, 2, 3, 4]
NAMES = ["1", "g5", "g1", "g2", "g3"]
NC = len(CODES)
TCODES = [c | 8 for c in CODES]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    import paper_2609_37049_amd as d
    d.lib()
    return d


@pytest.mark.timeout(900)
def test_precision_loops_16x16x16x32_one_timeslice(disco):
    """Partial loops (eigenvector index i < 2 for D, i < 4 for D_Lambda on the
    4^3 x 8 domains, the latter solved packed with the other three timeslices
    of its packing set) on one timeslice of the precision workload."""
    pre = synth.PRESETS["prec_16x16x16x32"]
    dims = pre.dims
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    U = synth.gauge_field(dims, pre.eps, pre.seed)
    A = oracle.clover(U, dims, pre.kappa, pre.csw)
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(pre.kappa, pre.csw)
    Vn = synth.random_colour_vectors(Lt, 4, Vs, 401)
    cut = synth.tiling_cuts(dims, pre.block)
    dom = ctx.domains(cut)
    t0 = 9
    layer = pre.block[3]
    pack = sum(1 << ((t0 + layer * k) % Lt) for k in range(Lt // layer))
    P = ctx.params(method=disco.BICGSTAB_RU, tol=1e-12, inner_prec=disco.BF16, rhs_block=64)
    rows = []
    for nv, c, dmn, msk in ((2, None, None, 1 << t0), (4, cut, dom, pack)):
        Vg = ctx.dev(np.ascontiguousarray(Vn[:, :nv]))
        tau = ctx.dev(np.zeros((Lt, nv, 4, nv, 4), dtype=np.complex128))
        agg = ctx.perambulators_tt(Vg, msk, P, tau, dmn)
        assert agg.true_rel_residual <= 1e-12
        L = ctx.loops(tau, CODES + TCODES).cpu().numpy()[:, t0]
        tau_o = np.zeros((nv, 4, nv, 4), dtype=np.complex128)
        for i in range(nv):
            X = [oracle.cgnr(U, A, dims, BC, pre.kappa, oracle.source(Vn, dims, t0, i, a), c, 1e-13)[0]
                 for a in range(4)]
            tau_o[:, :, i, :] = oracle.project(Vn[:, :nv], dims, np.stack(X), t0)
        L_o = oracle.loops(tau_o[None], CODES + TCODES)[:, 0]
        err = np.abs(L - L_o) / np.abs(L_o)
        rows.append(("D" if c is None else "D_Lambda", nv, err))
        assert err.max() <= 1e-10, (c is not None, err)
    _say("| operator | eigenvectors | " + " | ".join(NAMES) + " |")
    _say("|---|---|" + "---|" * NC)
    for op, nv, err in rows:
        _say("| %s | i < %d | %s |" % (op, nv, " | ".join("%.1e" % e for e in err[:NC])))


def _oracle_tau_tt(U, A, dims, kappa, Vo, cut, workers=8):
    """tau(t,t) of every timeslice from the oracle's CGNR solves (to 1e-13), the
    independent solves spread over a few host threads (each call releases the
    interpreter and runs its own small OpenMP team)."""
    from concurrent.futures import ThreadPoolExecutor
    T, nv = dims[3], Vo.shape[1]
    tau = np.empty((T, nv, 4, nv, 4), dtype=np.complex128)

    def one(job):
        t, i = job
        oracle.set_threads(2)
        X = [oracle.cgnr(U, A, dims, BC, kappa, oracle.source(Vo, dims, t, i, a), cut, 1e-13)[0] for a in range(4)]
        tau[t, :, :, i, :] = oracle.project(Vo, dims, np.stack(X), t)

    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(one, [(t, i) for t in range(T) for i in range(nv)]))
    return tau


@pytest.mark.timeout(900)
def test_precision_correlators_4x4x4x16_every_timeslice(disco):
    """Loops on every timeslice and the full, factorised and subtracted
    correlators at every separation, on a lattice where the oracle solves all
    of them: 4^3 x 16, Nv = 4 Laplacian eigenvectors of the oracle (3 APE
    steps), 2^3 x 4 domains (four temporal layers, four timeslices per packed
    solve)."""
    dims = (4, 4, 4, 16)
    kappa, csw = 0.124, 1.2
    T = dims[3]
    U = synth.gauge_field(dims, 0.3, 41)
    A = oracle.clover(U, dims, kappa, csw)
    Vo, _ = oracle.laplace_eigvecs(oracle.ape_smear(U, dims, 0.5, 3), dims, 4)
    cut = synth.tiling_cuts(dims, (2, 2, 2, 4))
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    ctx.clover_setup(kappa, csw)
    dom = ctx.domains(cut)
    P = ctx.params(method=disco.BICGSTAB_RU, tol=1e-12, inner_prec=disco.BF16, rhs_block=64)
    Vg = ctx.dev(Vo)
    Lf, _, a1 = ctx.loops_distill(Vg, CODES + TCODES, P)
    Lb, _, a2 = ctx.loops_distill(Vg, CODES + TCODES, P, dom)
    assert max(a1.true_rel_residual, a2.true_rel_residual) <= 1e-12
    Lf, Lb = Lf.cpu().numpy(), Lb.cpu().numpy()
    _say("oracle solves on 4x4x4x16 ...")
    tf = _oracle_tau_tt(U, A, dims, kappa, Vo, None)
    tb = _oracle_tau_tt(U, A, dims, kappa, Vo, cut)
    Lf_o, Lb_o = oracle.loops(tf, CODES + TCODES), oracle.loops(tb, CODES + TCODES)
    loop_err = {}
    for g in range(2 * NC):
        for name, La, Lr in (("D", Lf[g], Lf_o[g]), ("D_Lambda", Lb[g], Lb_o[g])):
            e = np.abs(La - Lr) / np.abs(Lr).max()
            loop_err[(name, g)] = e
            assert e.max() <= 1e-10, (name, g, e.max())
    corr_err = {}
    for g in range(NC):
        C, Cf, dC, _ = [x.cpu().numpy() for x in ctx.correlator(*[ctx.dev(v[None]) for v in (
            Lf[g], Lf[NC + g], Lb[g], Lb[NC + g])])]
        rC, rCf, rdC, _ = oracle.correlator(Lf_o[g][None], Lf_o[NC + g][None], Lb_o[g][None], Lb_o[NC + g][None])
        floor = 64 * np.finfo(float).eps * max(np.abs(Lf_o[g]).max(), np.abs(Lb_o[g]).max()) ** 2
        for name, got, ref in (("C", C, rC), ("C_fact", Cf, rCf), ("dC", dC, rdC)):
            e = np.abs(got - ref) / np.abs(ref).max()
            corr_err[(name, g)] = e
            assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max() + floor, (name, NAMES[g])
    _say("loops, max over t of |dL(t)| / max over t |L_ref| (D, D_Lambda):")
    _say("| channel | D | D_Lambda |")
    _say("|---|---|---|")
    for g in range(NC):
        _say("| %s | %.1e | %.1e |" % (NAMES[g], loop_err[("D", g)].max(), loop_err[("D_Lambda", g)].max()))
    for name in ("C", "dC"):
        _say("%s: |d%s(dt)| / max |%s_ref| per separation dt" % (name, name, name))
        _say("| dt | " + " | ".join(NAMES) + " |")
        _say("|---|" + "---|" * NC)
        for dt in range(T):
            _say("| %d | %s |" % (dt, " | ".join("%.1e" % corr_err[(name, g)][dt] for g in range(NC))))
