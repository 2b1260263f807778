"""GPU parity of the distillation chain against the FP64 oracle: APE smearing,
the covariant Laplacian and its eigenpairs, the perambulator projection on
matrix cores, loops, correlators, and end-to-end full and subtracted
correlators (with multi-site packing of the block solves)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from lattice_fixtures import unit_field, coords, momenta

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
CODES = [0, 1, 2, 3, 4]
TCODES = [c | 8 for c in CODES]   # the loops of Gamma~ = gamma_4 Gamma^+ gamma_4
NC = len(CODES)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def disco():
    import paper_2609_37049_amd as d
    d.lib()
    return d


def _ctx(disco, dims, U, kappa=None, csw=None):
    ctx = disco.Context(dims, BC)
    ctx.gauge_set(U)
    if kappa is not None:
        ctx.clover_setup(kappa, csw)
    return ctx


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_ape_parity(disco):
    dims = (4, 6, 4, 3)
    U = synth.gauge_field(dims, 0.4, 3)
    ctx = _ctx(disco, dims, U)
    ctx.ape_smear(3, 0.5)
    S = ctx.smeared_get().cpu().numpy()
    ref = oracle.ape_smear(U, dims, 0.5, 3)
    assert np.abs(S - ref).max() < 1e-13


def test_laplace_apply_parity(disco):
    dims = (5, 4, 6, 3)
    U = synth.gauge_field(dims, 0.5, 4)
    ctx = _ctx(disco, dims, U)
    V = int(np.prod(dims))
    rng = np.random.default_rng(1)
    y = rng.standard_normal((3, V, 3)) + 1j * rng.standard_normal((3, V, 3))
    out = ctx.laplace_apply(ctx.dev(y)).cpu().numpy()
    for k in range(3):
        assert _rel(out[k], oracle.laplace(U, dims, y[k])) < 1e-14


@pytest.mark.parametrize("dims,nv,steps", [((4, 4, 4, 4), 4, 0), ((6, 4, 4, 3), 10, 2), ((8, 8, 8, 2), 24, 1)])
def test_eigvecs_parity(disco, dims, nv, steps):
    _say("eigvecs", dims, nv)
    U = synth.gauge_field(dims, 0.3, 5)
    ctx = _ctx(disco, dims, U)
    if steps:
        ctx.ape_smear(steps, 0.5)
    Us = oracle.ape_smear(U, dims, 0.5, steps) if steps else U
    Vg, lam = ctx.laplace_eigvecs(nv, 1e-12)
    Vg = Vg.cpu().numpy()
    Vo, lo = oracle.laplace_eigvecs(Us, dims, nv)
    assert np.abs(lam - lo).max() < 1e-10
    T = dims[3]
    Vs = Vg.shape[2]
    for t in range(T):
        A = Vg[t].reshape(nv, -1)
        B = Vo[t].reshape(nv, -1)
        assert np.abs(np.conj(A) @ A.T - np.eye(nv)).max() < 1e-12
        # same spanned space (phases and rotations inside a cluster are free)
        assert np.abs(A.T @ np.conj(A) - B.T @ np.conj(B)).max() < 1e-8


def test_eigvecs_on_chosen_timeslices(disco):
    """Eigenpairs on a few timeslices only equal those of the all-timeslice
    solve there (eigenvalues, and the projector onto the eigenvectors, which
    does not depend on their phases), on smeared links."""
    dims = (6, 4, 4, 6)
    U = synth.gauge_field(dims, 0.4, 17)
    ctx = _ctx(disco, dims, U)
    ctx.ape_smear(2, 0.5)
    Vg, lam = ctx.laplace_eigvecs(5, 1e-13)
    ts = [4, 1, 5]
    Vs_, lam_s = ctx.laplace_eigvecs_slices(5, ts, 1e-13)
    Vg, Vs_ = Vg.cpu().numpy(), Vs_.cpu().numpy()
    for k, t in enumerate(ts):
        assert np.abs(lam_s[k] - lam[t]).max() < 1e-11
        A = Vg[t].reshape(5, -1)
        B = Vs_[k].reshape(5, -1)
        assert np.abs(A.T @ np.conj(A) - B.T @ np.conj(B)).max() < 1e-9
    with pytest.raises(disco.DiscoError):
        ctx.laplace_eigvecs_slices(5, [1, 1])


def test_perambulator_parity(disco):
    """Same V and X on both sides: tau = V^+ X at several sink timeslices (FP64 MFMA)."""
    dims = (6, 4, 4, 5)
    U = synth.gauge_field(dims, 0.4, 6)
    ctx = _ctx(disco, dims, U)
    Vo, _ = oracle.laplace_eigvecs(U, dims, 7)
    V = int(np.prod(dims))
    for nsrc in (1, 5, 16):
        X = synth.random_spinor(V, nsrc, 7 + nsrc)
        t_snk = [0, 3, 4]
        tau = ctx.perambulator(ctx.dev(Vo), ctx.dev(X), t_snk).cpu().numpy()
        for k, t in enumerate(t_snk):
            ref = oracle.project(Vo, dims, X, t)
            assert _rel(tau[k], ref) < 1e-14


def test_loops_parity(disco):
    rng = np.random.default_rng(8)
    T, nv = 5, 6
    tau = rng.standard_normal((T, nv, 4, nv, 4)) + 1j * rng.standard_normal((T, nv, 4, nv, 4))
    w = rng.random((T, nv))
    ctx = disco.Context((2, 2, 2, T), BC)
    for ww in (None, w):
        L = ctx.loops(ctx.dev(tau), CODES, None if ww is None else ctx.dev(ww)).cpu().numpy()
        ref = oracle.loops(tau, CODES, ww)
        assert _rel(L, ref) < 1e-14


def test_tilde_loops_parity(disco):
    """Loop codes with the tilde flag give the loops of gamma_4 Gamma^+ gamma_4,
    formed in the library's loop kernel (the oracle forms the matrix product)."""
    rng = np.random.default_rng(18)
    T, nv = 6, 5
    tau = rng.standard_normal((T, nv, 4, nv, 4)) + 1j * rng.standard_normal((T, nv, 4, nv, 4))
    w = rng.random((T, nv))
    ctx = disco.Context((2, 2, 2, T), BC)
    for ww in (None, w):
        L = ctx.loops(ctx.dev(tau), CODES + TCODES, None if ww is None else ctx.dev(ww)).cpu().numpy()
        ref = oracle.loops(tau, CODES + TCODES, ww)
        assert _rel(L, ref) < 1e-14
        # +L for 1, -L for gamma_5 and gamma_k (a consequence, checked on the GPU's output)
        for g in range(NC):
            s = 1.0 if CODES[g] == 0 else -1.0
            assert np.abs(L[NC + g] - s * L[g]).max() <= 1e-14 * np.abs(L[g]).max()
    with pytest.raises(disco.DiscoError):
        ctx.loops(ctx.dev(tau), [16])


@pytest.mark.parametrize("vev_mode", [0, 1])
def test_correlator_parity(disco, vev_mode):
    rng = np.random.default_rng(9)
    ncfg, T = 6, 8
    mk = lambda: rng.standard_normal((ncfg, T)) + 1j * rng.standard_normal((ncfg, T))
    Lf, Ltf = mk(), mk()
    Lb, Ltb = Lf + 0.1 * mk(), Ltf + 0.1 * mk()
    ctx = disco.Context((2, 2, 2, T), BC)
    for y0s in (None, [1, 4]):
        C, Cf, dC, four = [a.cpu().numpy() for a in ctx.correlator(ctx.dev(Lf), ctx.dev(Ltf), ctx.dev(Lb),
                                                                    ctx.dev(Ltb), y0s, vev_mode)]
        rC, rCf, rdC, rfour = oracle.correlator(Lf, Ltf, Lb, Ltb, y0s, vev_mode)
        for a, b in ((C, rC), (Cf, rCf), (dC, rdC), (four, rfour)):
            assert np.abs(a - b).max() < 1e-13 * max(1.0, np.abs(rC).max())


@pytest.fixture(scope="module")
def plain_oracle():
    """Oracle loops for the plain FP64 workload (4^4, Nv=4, 2^4 domains)."""
    pre = synth.PRESETS["plain_4x4x4x4"]
    dims = pre.dims
    U = synth.gauge_field(dims, pre.eps, pre.seed)
    A = oracle.clover(U, dims, pre.kappa, pre.csw)
    Us = oracle.ape_smear(U, dims, pre.ape_alpha, pre.ape_steps) if pre.ape_steps else U
    Vo, _ = oracle.laplace_eigvecs(Us, dims, pre.nv)
    cut = synth.tiling_cuts(dims, pre.block)
    T = dims[3]
    tau_f = np.stack([oracle.perambulator_tt(U, A, dims, BC, pre.kappa, Vo, t) for t in range(T)])
    tau_b = np.stack([oracle.perambulator_tt(U, A, dims, BC, pre.kappa, Vo, t, cut=cut) for t in range(T)])
    return (pre, U, A, Vo, cut, oracle.loops(tau_f, CODES + TCODES), oracle.loops(tau_b, CODES + TCODES), tau_f,
            tau_b)


@pytest.mark.parametrize("method,blk", [("CGNR_F64", 8), ("BICGSTAB_DC", 8), ("BICGSTAB_RU", 8), ("BICGSTAB_RU", 5)])
def test_end_to_end_plain_workload(disco, plain_oracle, method, blk):
    """4^4 plain workload: the GPU computes its own eigenvectors, solves to 1e-12
    (full operator and packed block solves), and its loops and full, factorised
    and subtracted correlators agree with the oracle's to 1e-10.  With reliable
    updates the lanes take the sources of every timeslice from one queue (a
    block of 5 lanes does not divide the 16 sources of a timeslice)."""
    pre, U, A, Vo, cut, Lf_o, Lb_o, tau_f_o, tau_b_o = plain_oracle
    dims = pre.dims
    _say("end-to-end", method, blk)
    ctx = _ctx(disco, dims, U, pre.kappa, pre.csw)
    if pre.ape_steps:
        ctx.ape_smear(pre.ape_steps, pre.ape_alpha)
    Vg, _ = ctx.laplace_eigvecs(pre.nv, 1e-13)
    dom = ctx.domains(cut)
    P = ctx.params(method=getattr(disco, method), tol=1e-12, inner_prec=disco.F32, rhs_block=blk)
    Lf, tf, st = ctx.loops_distill(Vg, CODES + TCODES, P, None, want_tau=True)
    Lb, tb, stb = ctx.loops_distill(Vg, CODES + TCODES, P, dom, want_tau=True)
    # packing: 2 temporal layers -> half as many block solves as logical sources
    assert ctx.last_solves() == 4 * pre.nv * dims[3] // 2
    Lf, Lb = Lf.cpu().numpy(), Lb.cpu().numpy()
    for g in range(2 * NC):
        for La, Lr in ((Lf[g], Lf_o[g]), (Lb[g], Lb_o[g])):
            err = np.abs(La - Lr).max() / max(np.abs(Lr).max(), 1e-300)
            assert err < 1e-10, (g, err)
    # correlators per channel (one configuration: translation-averaged VEV), the
    # source side taking the library's loops of Gamma~
    for g in range(NC):
        args = [ctx.dev(v[None]) for v in (Lf[g], Lf[NC + g], Lb[g], Lb[NC + g])]
        C, Cf, dC, four = [a.cpu().numpy() for a in ctx.correlator(*args)]
        rC, rCf, rdC, _ = oracle.correlator(Lf_o[g][None], Lf_o[NC + g][None], Lb_o[g][None], Lb_o[NC + g][None])
        # 1e-10 of the correlator, plus the FP64 rounding floor of the VEV-subtracted
        # products <L Lt> - <L><Lt> (both sides hit it when C is far below |L|^2)
        floor = 64 * np.finfo(float).eps * max(np.abs(Lf_o[g]).max(), np.abs(Lb_o[g]).max()) ** 2
        tol = 1e-10 * np.abs(rC).max() + floor
        assert np.abs(C - rC).max() <= tol
        assert np.abs(Cf - rCf).max() <= tol
        assert np.abs(dC - rdC).max() <= tol
        assert np.abs(four.sum(axis=0) - C).max() <= floor


def test_single_domain_block_loops_equal_full(disco):
    dims = (4, 4, 2, 4)
    U = synth.gauge_field(dims, 0.3, 13)
    ctx = _ctx(disco, dims, U, 0.12, 1.0)
    Vg, _ = ctx.laplace_eigvecs(3, 1e-12)
    dom = ctx.domains(np.zeros((4, 4), dtype=np.uint8))
    P = ctx.params(method=disco.CGNR_F64, tol=1e-12, rhs_block=12)
    Lf, _, _ = ctx.loops_distill(Vg, CODES, P, None)
    Lb, _, _ = ctx.loops_distill(Vg, CODES, P, dom)
    assert np.abs(Lf.cpu().numpy() - Lb.cpu().numpy()).max() < 1e-10 * np.abs(Lf.cpu().numpy()).max()


def test_uneven_domains_packing_exact(disco):
    """Uneven temporal layers (offset tiling): packed block loops equal the
    oracle's unpacked ones."""
    dims = (4, 4, 4, 6)
    U = synth.gauge_field(dims, 0.3, 14)
    kappa, csw = 0.12, 1.2
    ctx = _ctx(disco, dims, U, kappa, csw)
    A = oracle.clover(U, dims, kappa, csw)
    cut = synth.offset_tiling_cuts(dims, (4, 4, 4, 4))  # t layers of extent 2, 4 (wrapped offset)
    dom = ctx.domains(cut)
    Vo, _ = oracle.laplace_eigvecs(U, dims, 2)
    P = ctx.params(method=disco.BICGSTAB_DC, tol=1e-12, rhs_block=8)
    Lb, _, _ = ctx.loops_distill(ctx.dev(Vo), CODES, P, dom)
    tau = np.stack([oracle.perambulator_tt(U, A, dims, BC, kappa, Vo, t, cut=cut) for t in range(dims[3])])
    ref = oracle.loops(tau, CODES)
    assert np.abs(Lb.cpu().numpy() - ref).max() < 1e-10 * np.abs(ref).max()


def test_free_field_loops_full_size(disco):
    """16^3 x 32 at U = 1 with plane-wave distillation vectors: the end-to-end
    GPU loops equal the momentum-space closed form
    L_Gamma(t) = sum_(k,c) (1/Lt) sum_p4 Tr[Gamma D(k,p4)^-1]."""
    dims = (16, 16, 16, 32)
    kappa = 0.12
    _say("free field full size")
    U = unit_field(dims)
    ctx = _ctx(disco, dims, U, kappa, 1.0)
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    X = coords(dims)[:Vs, :3]
    ks = [(0.0, 0.0, 0.0), (2 * np.pi / 16, 0.0, 0.0), (0.0, 2 * np.pi * 3 / 16, 2 * np.pi / 16)]
    vecs = []
    for k in ks:
        ph = np.exp(1j * (X @ np.asarray(k))) / np.sqrt(Vs)
        for c in range(3):
            v = np.zeros((Vs, 3), dtype=np.complex128)
            v[:, c] = ph
            vecs.append(v)
    Vt = np.broadcast_to(np.stack(vecs), (Lt, len(vecs), Vs, 3)).copy()
    P = ctx.params(method=disco.BICGSTAB_DC, tol=1e-11, inner_prec=disco.F32, rhs_block=12)
    L, _, st = ctx.loops_distill(ctx.dev(Vt), CODES, P, None)
    L = L.cpu().numpy()
    g = [oracle.gamma(m) for m in range(4)]
    p4s = momenta(dims, BC)[3]
    for ci, c in enumerate(CODES):
        gm = oracle.channel_matrix(c)
        ref = 0j
        for k in ks:
            for p4 in p4s:
                p = list(k) + [p4]
                M = 1 - 2 * kappa * sum(np.cos(p))
                S = (M * np.eye(4) - 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))) / (
                    M ** 2 + 4 * kappa ** 2 * sum(np.sin(p) ** 2))
                ref += 3 * np.trace(gm @ S) / len(p4s)
        assert np.abs(L[ci] - ref).max() <= 1e-9 * max(abs(ref), 1.0), (c, L[ci][:3], ref)


def test_full_size_eigvecs(disco):
    """16^3 x 32 with 5 APE steps, Nv = 32: residuals, orthonormality, and the
    eigenvalues of two timeslices against the oracle (ARPACK on its Laplacian)."""
    pre = synth.PRESETS["prec_16x16x16x32"]
    dims = pre.dims
    _say("full-size eigvecs")
    U = synth.gauge_field(dims, pre.eps, pre.seed)
    ctx = _ctx(disco, dims, U)
    ctx.ape_smear(pre.ape_steps, pre.ape_alpha)
    Vg, lam = ctx.laplace_eigvecs(pre.nv, 1e-10)
    assert np.all(np.diff(lam, axis=1) >= -1e-12)
    Us = ctx.smeared_get().cpu().numpy()
    Uo = oracle.ape_smear(U, dims, pre.ape_alpha, pre.ape_steps)
    assert np.abs(Us - Uo).max() < 1e-12
    import scipy.sparse.linalg as sla
    Vs = dims[0] * dims[1] * dims[2]
    V = Vs * dims[3]
    Vn = Vg.cpu().numpy()
    d1 = (dims[0], dims[1], dims[2], 1)
    for t in (0, 17):
        Ut = np.ascontiguousarray(Uo[t * Vs:(t + 1) * Vs])

        def mv(y, Ut=Ut):
            return oracle.laplace(Ut, d1, y.reshape(Vs, 3)).reshape(-1)
        op = sla.LinearOperator((3 * Vs, 3 * Vs), matvec=mv, dtype=np.complex128)
        w = np.sort(sla.eigsh(op, k=pre.nv, which="SA", tol=1e-12, return_eigenvectors=False))
        assert np.abs(w - lam[t]).max() < 1e-8
        A = Vn[t].reshape(pre.nv, -1)
        assert np.abs(np.conj(A) @ A.T - np.eye(pre.nv)).max() < 1e-11


@pytest.mark.parametrize("delta", [1, 3, 5])
def test_slab_schedule_loops(disco, delta):
    """The paper's regions: a temporal slab of width delta centred on every
    operator time x0, solved set by set with multi-site sources on the GPU,
    against the oracle solving every x0 on its own; plus the Gaussian-profiled
    loops from the same perambulators (weights from each side's own
    eigenvalues)."""
    dims = (4, 4, 4, 8)
    kappa, csw = 0.12, 1.0
    codes = [disco.G_1, disco.G_5, disco.G_X, disco.G_Y, disco.G_Z]
    U = synth.gauge_field(dims, 0.3, 91)
    A = oracle.clover(U, dims, kappa, csw)
    Us = oracle.ape_smear(U, dims, 0.5, 2)
    Vo, lam_o = oracle.laplace_eigvecs(Us, dims, 4)
    Lo, tau_o = oracle.slab_loops(U, A, dims, BC, kappa, Vo, delta, codes)
    ctx = _ctx(disco, dims, U, kappa, csw)
    ctx.ape_smear(2, 0.5)
    Vg, lam_g = ctx.laplace_eigvecs(4, 1e-13)
    sets = ctx.slab_sets(delta)
    T = dims[3]
    assert sorted(sum(([t for t in range(T) if (m >> t) & 1] for m in sets), [])) == list(range(T))
    P = ctx.params(method=disco.BICGSTAB_DC, tol=1e-12, inner_prec=disco.F32, rhs_block=8)
    L, tau_g, st = ctx.loops_slab(Vg, codes, delta, P, want_tau=True)
    _say("  slab delta %d: %d sets, %d solves, worst residual %.2e" % (delta, len(sets), ctx.last_solves(),
                                                                       st.true_rel_residual))
    assert ctx.last_solves() == len(sets) * 16
    L = L.cpu().numpy()
    for g in range(len(codes)):
        err = np.abs(L[g] - Lo[g]).max() / np.abs(Lo[g]).max()
        assert err < 1e-10, (g, err)
    for omega in (0.05, 0.287):
        wg = ctx.profile_weights(lam_g, omega)
        wo = oracle.profile_weights(lam_o, omega)
        Lw = ctx.loops(tau_g, codes, ctx.dev(wg)).cpu().numpy()
        Lwo = oracle.loops(tau_o, codes, wo)
        for g in range(len(codes)):
            err = np.abs(Lw[g] - Lwo[g]).max() / max(np.abs(Lwo[g]).max(), 1e-300)
            assert err < 1e-9, (omega, g, err)


@pytest.mark.parametrize("delta", [3, 5])
def test_open_time_slab_schedule_loops(disco, delta):
    """The paper's open time boundary: slabs clipped at t = 0 and T-1, the wrap
    face cut in every partition, sets packed by distance on the open line;
    slab loops against the oracle solving every x0 on its own, and the loops
    of the full open-boundary operator (domains cutting only the wrap face)
    against the oracle's; plus C^NR spliced over two widths by the library
    against the oracle's rule on the same correlators."""
    dims = (4, 4, 4, 8)
    kappa, csw = 0.12, 1.0
    T = dims[3]
    U = synth.gauge_field(dims, 0.3, 94)
    A = oracle.clover(U, dims, kappa, csw)
    Vo, _ = oracle.laplace_eigvecs(oracle.ape_smear(U, dims, 0.5, 2), dims, 3)
    Lo, _ = oracle.slab_loops(U, A, dims, BC, kappa, Vo, delta, CODES + TCODES, open_time=True)
    ocut = oracle.open_time_cut(dims)
    tau_fo = np.stack([oracle.perambulator_tt(U, A, dims, BC, kappa, Vo, t, cut=ocut) for t in range(T)])
    Lfo = oracle.loops(tau_fo, CODES + TCODES)
    ctx = _ctx(disco, dims, U, kappa, csw)
    Vg = ctx.dev(Vo)
    sets = ctx.slab_sets(delta, open_time=True)
    assert sorted(sum(([t for t in range(T) if (m >> t) & 1] for m in sets), [])) == list(range(T))
    for m in sets:   # disjoint on the open line
        xs = [t for t in range(T) if (m >> t) & 1]
        assert all(b - a >= delta for a, b in zip(xs, xs[1:]))
    P = ctx.params(method=disco.BICGSTAB_RU, tol=1e-12, inner_prec=disco.F32, rhs_block=8)
    L, _, st = ctx.loops_slab(Vg, CODES + TCODES, delta, P, open_time=True)
    assert ctx.last_solves() == len(sets) * 12
    wrap = np.zeros((4, max(dims)), dtype=np.uint8)
    wrap[3, T - 1] = 1   # the open time boundary: only the face between T-1 and 0
    Lf, _, _ = ctx.loops_distill(Vg, CODES + TCODES, P, ctx.domains(wrap))
    L, Lf = L.cpu().numpy(), Lf.cpu().numpy()
    for g in range(2 * NC):
        for La, Lr in ((L[g], Lo[g]), (Lf[g], Lfo[g])):
            err = np.abs(La - Lr).max() / np.abs(Lr).max()
            assert err < 1e-10, (delta, g, err)
    # C^NR over widths 1 and delta (library splice of the library's correlators vs
    # the oracle's rule on the oracle's), Gamma = gamma_5
    L1, _, _ = ctx.loops_slab(Vg, CODES + TCODES, 1, P, open_time=True)
    L1 = L1.cpu().numpy()
    L1o, _ = oracle.slab_loops(U, A, dims, BC, kappa, Vo, 1, CODES + TCODES, open_time=True)
    g = 1
    dC = [ctx.correlator(*[ctx.dev(v[None]) for v in (Lf[g], Lf[NC + g], Lb[g], Lb[NC + g])])[2].cpu().numpy()
          for Lb in (L1, L)]
    dCo = [oracle.correlator(Lfo[g][None], Lfo[NC + g][None], Lbo[g][None], Lbo[NC + g][None])[2]
           for Lbo in (L1o, Lo)]
    rng = np.random.default_rng(95)
    Cc = rng.standard_normal(T) + 1j * rng.standard_normal(T)   # a stand-in connected correlator, both sides
    got = ctx.nr_splice(Cc, np.stack(dC), [1, delta])
    ref = oracle.nr_splice(Cc, np.stack(dCo), [1, delta])
    assert np.array_equal(np.isnan(got), np.isnan(ref)) and np.isnan(got[:2]).all()
    ok = ~np.isnan(ref)
    scale = np.abs(ref[ok]).max()
    assert np.abs(got[ok] - ref[ok]).max() <= 1e-10 * scale


@pytest.mark.parametrize("method,blk", [("BICGSTAB_DC", 12), ("BICGSTAB_RU", 5)])
def test_connected_correlator_and_noise_reduced_estimator(disco, method, blk):
    """All-to-all perambulators on the GPU and the connected contraction (the
    sink-to-source direction from gamma_5-hermiticity) against the oracle,
    which takes both directions from direct solves; C^NR = C^(c) + dC and the
    effective mass from the library's helper."""
    dims = (4, 4, 4, 8)
    kappa, csw = 0.12, 1.0
    codes = [disco.G_1, disco.G_5, disco.G_X]
    U = synth.gauge_field(dims, 0.3, 111)
    A = oracle.clover(U, dims, kappa, csw)
    Us = oracle.ape_smear(U, dims, 0.5, 2)
    Vo, lam_o = oracle.laplace_eigvecs(Us, dims, 3)
    T = dims[3]
    tau_o = np.stack([oracle.perambulator_all(U, A, dims, BC, kappa, Vo, ts) for ts in range(T)])
    Co = oracle.connected(tau_o, codes)
    wo = oracle.profile_weights(lam_o, 0.287)
    Cow = oracle.connected(tau_o, codes, wo, y0s=[0, 3, 5])
    ctx = _ctx(disco, dims, U, kappa, csw)
    ctx.ape_smear(2, 0.5)
    Vg, lam_g = ctx.laplace_eigvecs(3, 1e-13)
    P = ctx.params(method=getattr(disco, method), tol=1e-12, inner_prec=disco.F32, rhs_block=blk)
    tau_g, st = ctx.perambulators_all(Vg, P)
    assert ctx.last_solves() == T * 12
    C = ctx.connected(tau_g, codes).cpu().numpy()
    Cw = ctx.connected(tau_g, codes, ctx.dev(ctx.profile_weights(lam_g, 0.287)), y0s=[0, 3, 5]).cpu().numpy()
    for g in range(len(codes)):
        for a, r in ((C[g], Co[g]), (Cw[g], Cow[g])):
            err = np.abs(a - r).max() / np.abs(r).max()
            _say("  connected channel %d: rel error %.2e" % (codes[g], err))
            assert err < 1e-10
    # the pseudoscalar connected correlator is real and positive
    assert np.abs(C[1].imag).max() < 1e-10 * np.abs(C[1].real).max()
    assert (C[1].real > 0).all()
    # noise-reduced estimator: connected + subtracted disconnected
    dom = ctx.domains(synth.tiling_cuts(dims, (4, 4, 4, 4)))
    Lf, _, _ = ctx.loops_distill(Vg, [disco.G_5], P)
    Lb, _, _ = ctx.loops_distill(Vg, [disco.G_5], P, dom)
    _, _, dC, _ = ctx.correlator(Lf, -Lf, Lb, -Lb)
    CNR = C[1] + dC.cpu().numpy()
    assert np.isfinite(CNR).all()
    m = ctx.effective_mass(C[1].real[: T // 2 + 1])
    ref = np.log(C[1].real[: T // 2] / C[1].real[1: T // 2 + 1])
    assert np.abs(m - ref).max() < 1e-14


def test_bench_configuration_perambulators_sampled(disco):
    """The benchmark's solver configuration on the full 16^3 x 32 workload:
    BF16-stored BiCGStab with reliable updates, 64 lanes fed from one queue,
    projections of the handed-over lanes; D on one timeslice (128 sources
    through 64 lanes) and D_Lambda on one packing set (four timeslices per
    solve).  Both sides take the same seeded smearing vectors (the projection
    V^+ D^-1 V is defined for any V; the Laplacian eigenvectors are checked on
    their own), and sampled columns tau(t,t)[:, :, i, alpha] are compared with
    the oracle's own CGNR solves of those sources (D_Lambda unpacked, one
    timeslice at a time).

    Tolerance: both sides stop at a true relative residual (1e-10 here, 1e-11
    for the oracle), so |tau - tau_ref| <= |D^-1| 1e-10 with unit sources; the
    bound 1e-7 of max|tau_ref| allows |D^-1| up to 1e3.  Any wrong lane, source
    or sink timeslice gives an error of order one."""
    pre = synth.PRESETS["prec_16x16x16x32"]
    dims = pre.dims
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    nv = pre.nv
    _say("bench configuration, sampled perambulators")
    U = synth.gauge_field(dims, pre.eps, pre.seed)
    ctx = _ctx(disco, dims, U, pre.kappa, pre.csw)
    Vn = synth.random_colour_vectors(Lt, nv, Vs, 77)
    Vev = ctx.dev(Vn)
    cut = synth.tiling_cuts(dims, pre.block)
    dom = ctx.domains(cut)
    P = ctx.params(method=disco.BICGSTAB_RU, tol=1e-10, inner_prec=disco.BF16, rhs_block=64)
    t0 = 5
    layer = pre.block[3]
    tau_f = ctx.dev(np.zeros((Lt, nv, 4, nv, 4), dtype=np.complex128))
    tau_b = ctx.dev(np.zeros((Lt, nv, 4, nv, 4), dtype=np.complex128))
    ctx.perambulators_tt(Vev, 1 << t0, P, tau_f)
    assert ctx.last_solves() == 4 * nv
    pack = sum(1 << (t0 + layer * k) for k in range(Lt // layer))
    ctx.perambulators_tt(Vev, pack, P, tau_b, dom)
    assert ctx.last_solves() == 4 * nv   # four timeslices per packed solve
    tf, tb = tau_f.cpu().numpy(), tau_b.cpu().numpy()
    A = oracle.clover(U, dims, pre.kappa, pre.csw)
    for tau, c, ts in ((tf, None, (t0,)), (tb, cut, (t0, t0 + 2 * layer))):
        for t in ts:
            for i, a in ((0, 0), (nv - 1, 3)):
                x, it, rr = oracle.cgnr(U, A, dims, BC, pre.kappa, oracle.source(Vn, dims, t, i, a), c, 1e-11)
                ref = oracle.project(Vn, dims, x[None], t)[:, :, 0]
                err = np.abs(tau[t, :, :, i, a] - ref).max() / np.abs(ref).max()
                _say("  %s t=%d (i,alpha)=(%d,%d): %d oracle iterations, rel error %.2e" % (
                    "D_Lambda" if c is not None else "D", t, i, a, it, err))
                assert err < 1e-7
    # timeslices outside the masks are not written
    assert np.abs(tf[t0 + 1]).max() == 0 and np.abs(tb[t0 + 1]).max() == 0


def test_bench_shape_loops_and_correlators(disco):
    """The bench's loop and correlator calls at its 16^3 x 32 shape (T = 32,
    Nv = 32, the five channels and their Gamma~ loops from the library), on
    seeded perambulators given to both sides, against the oracle's traces and
    VEV-subtracted products."""
    T, nv = 32, 32
    rng = np.random.default_rng(78)
    mk = lambda: rng.standard_normal((T, nv, 4, nv, 4)) + 1j * rng.standard_normal((T, nv, 4, nv, 4))
    tf, tb = mk(), mk()
    tb = tf + 0.05 * tb
    ctx = disco.Context((2, 2, 2, T), BC)
    Lf = ctx.loops(ctx.dev(tf), CODES + TCODES).cpu().numpy()
    Lb = ctx.loops(ctx.dev(tb), CODES + TCODES).cpu().numpy()
    Lf_o = oracle.loops(tf, CODES + TCODES)
    Lb_o = oracle.loops(tb, CODES + TCODES)
    assert _rel(Lf, Lf_o) < 1e-13 and _rel(Lb, Lb_o) < 1e-13
    for g in range(NC):
        args = [ctx.dev(v[None]) for v in (Lf_o[g], Lf_o[NC + g], Lb_o[g], Lb_o[NC + g])]
        C, Cf, dC, four = [x.cpu().numpy() for x in ctx.correlator(*args)]
        rC, rCf, rdC, rfour = oracle.correlator(Lf_o[g][None], Lf_o[NC + g][None], Lb_o[g][None],
                                                Lb_o[NC + g][None])
        floor = 64 * np.finfo(float).eps * max(np.abs(Lf_o[g]).max(), np.abs(Lb_o[g]).max()) ** 2
        tol = 1e-10 * np.abs(rC).max() + floor
        for got, ref in ((C, rC), (Cf, rCf), (dC, rdC), (four, rfour)):
            assert np.abs(got - ref).max() <= tol, CODES[g]
        assert np.abs(four.sum(axis=0) - C).max() <= floor